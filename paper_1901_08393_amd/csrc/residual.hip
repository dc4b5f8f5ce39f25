// Weighted-residual error estimator of the primal P0 solution (Appendix A,
// eq. "residual:indicator"):
//
//   mu(T)^2 = diam(T) || grad_G (f - V Phi) ||^2_{L2(T)},   f = 1,
//
// with the residual evaluated in the discontinuous piecewise linears (the
// paper's remark on the estimator's cost: the P1 Galerkin operator gives the
// residual in P1).  On T the residual is replaced by its L2 projection onto
// the linear functions, whose gradient is constant.  With the first moments
//
//   m_k(T_i) = <V Phi, lambda_k>_{T_i}
//            = sum_j Phi_j (1/4pi) int_{T_i} lambda_k(x) int_{T_j} 1/|x-y| dy dx
//
// (lambda_k the barycentric coordinate of the k-th input vertex of T_i) the
// projection of 1 - V Phi is sum_k c_k lambda_k with c = M_T^{-1}(|T|/3 - m),
// M_T = |T| (1 + delta_kl) / 12; its constant part has no gradient, and
// grad lambda_k = n x e_k / (2|T|) with e_k = P_{k+2} - P_{k+1}, so
//
//   mu(T)^2 = diam(T) |T| |grad|^2 = 36 diam(T) |sum_k m_k e_k|^2 / |T|^3.
//
// The moments use the matrix's quadrature in FP64: the collapsed Gauss rule
// on both triangles for pairs that share no vertex (k_res_far: all ordered
// pairs, lanes own rows, the columns of a chunk are visited in order with
// uniform loads, touching columns skipped), the Sauter-Schwab-type rules
// with the linear weight for touching pairs (k_res_touch: one wavefront per
// pattern entry, on the canonical pair (min, max) so that both orders use the
// same points as the pair's matrix entry), and k_res_finish sums the chunks
// and the row's pattern entries in a fixed order.  ALU-bound like the
// assembly: N^2 Q^2 point pairs (all ordered pairs), each about ten FP64
// instructions and one inverse square root (instruction counters).
#include "bc_internal.h"

namespace bc {

// w_a lambda_k(a) of the collapsed rule's points: lambda = (1 - s - t, s, t)
// at (s, t) = (xi_a, xi_b (1 - xi_a)), weights w_a w_b (1 - xi_a).
struct ResRule {
  double wl[3][kQMax];
};

constexpr int kResTargetWG = 2048;  // workgroups of k_res_far aimed at (8 per CU)

// Column chunks of k_res_far for N elements: a function of N only, so the
// summation order (and the result) does not depend on the device.
inline int res_chunks(int64_t N) {
  const int64_t rows = (N + kWG - 1) / kWG;
  int64_t c = (kResTargetWG + rows - 1) / rows;
  const int64_t cmax = (N + 63) / 64;  // at least 64 columns per chunk
  if (c > cmax) c = cmax;
  if (c < 1) c = 1;
  return (int)c;
}

struct ResLayout {
  size_t part, tv, total;
  int C;
  ResLayout(int64_t N, int64_t nnz) {
    C = res_chunks(N);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    part = take(sizeof(double) * 3 * (size_t)C * (size_t)N);
    tv = take(sizeof(double) * 3 * (size_t)nnz);
    total = o;
  }
};

__device__ __forceinline__ double rsqrt64_res2(double x) {
  // hardware estimate and one Newton step, as in the FP64 far field: returns
  // y (3 - x y^2), twice the refined value (the caller halves the weight)
  const double y = __builtin_amdgcn_rsq(x);
  return y * __builtin_fma(-(x * y), y, 3.0);
}

// part[c][i][k] = sum_{j in chunk c, no vertex shared with i} Phi_j
//                 sum_a w_a lambda_k(a) sum_b W_b / |x_a - y_b|
template <int Q>
__global__ __launch_bounds__(kWG) void k_res_far(const double4 *__restrict__ qpA, const int4 *__restrict__ tri4,
                                                 const double *__restrict__ sigma, ResRule rr, int N, int chunk,
                                                 double *__restrict__ part) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  const bool iv = i < N;
  const int ii = iv ? i : N - 1;
  double xx[Q], xy[Q], xz[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double4 p = qpA[(size_t)ii * kQMax + a];
    xx[a] = p.x; xy[a] = p.y; xz[a] = p.z;
  }
  const int4 ti = tri4[ii];
  const int c = blockIdx.y;
  const int j0 = c * chunk, j1 = min(N, j0 + chunk);
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  for (int j = j0; j < j1; ++j) {  // j is the same in every lane: uniform loads
    const double4 *yb = qpA + (size_t)j * kQMax;
    double s[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) s[a] = 0.0;
#pragma unroll 4
    for (int b = 0; b < Q; ++b) {
      const double4 y = yb[b];
      const double hw = 0.5 * y.w;  // the Newton step's 1/2
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const double dx = xx[a] - y.x, dy = xy[a] - y.y, dz = xz[a] - y.z;
        s[a] = __builtin_fma(hw, rsqrt64_res2(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx))), s[a]);
      }
    }
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      t0 = __builtin_fma(rr.wl[0][a], s[a], t0);
      t1 = __builtin_fma(rr.wl[1][a], s[a], t1);
      t2 = __builtin_fma(rr.wl[2][a], s[a], t2);
    }
    const int4 tj = tri4[j];
    const bool touch = ti.x == tj.x || ti.x == tj.y || ti.x == tj.z || ti.y == tj.x || ti.y == tj.y ||
                       ti.y == tj.z || ti.z == tj.x || ti.z == tj.y || ti.z == tj.z;
    // touching pairs (the coincident one has r = 0) are the singular rules'
    t0 = touch ? 0.0 : t0;
    t1 = touch ? 0.0 : t1;
    t2 = touch ? 0.0 : t2;
    const double pj = sigma[j];
    acc0 = __builtin_fma(pj, t0, acc0);
    acc1 = __builtin_fma(pj, t1, acc1);
    acc2 = __builtin_fma(pj, t2, acc2);
  }
  if (iv) {
    double *o = part + ((size_t)c * N + i) * 3;
    o[0] = acc0; o[1] = acc1; o[2] = acc2;
  }
}

// tv[e][k] = moment k on T_i of the pattern entry e = (i, j) with the
// singular rule of the pair's order, scale (1/4pi)(2|T_p|)(2|T_q|) included; 0 for
// near entries (k_res_far covers them).  The rule runs on the canonical pair
// (p, q) = (min(i, j), max(i, j)); the linear weight is taken at the points
// of T_i: lambda = (1 - x1, x1 - x2, x2) on the canonical vertices of T_p,
// or (1 - y1, y1 - y2, y2) on those of T_q.
__global__ __launch_bounds__(kWG) void k_res_touch(const double *__restrict__ verts, const int4 *__restrict__ tri4,
                                                   const double4 *__restrict__ cen4, const double *__restrict__ area,
                                                   SSTable ss, const int32_t *__restrict__ prow,
                                                   const int32_t *__restrict__ pcol, const int32_t *__restrict__ pkind,
                                                   int64_t nnz, double *__restrict__ tv) {
  const int64_t e = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (e >= nnz) return;
  const int lane = threadIdx.x & 63;
  const int i = prow[e], j = pcol[e], kind = pkind[e];
  double mc0 = 0.0, mc1 = 0.0, mc2 = 0.0;  // moments on the canonical vertices of T_i
  int slot[3] = {0, 1, 2};
  double scale = 0.0;
  if (kind != kNear) {
    const int p = min(i, j), q = max(i, j);
    const bool first = i == p;  // the coincident pair takes the x points
    const TouchOrder o = touch_order(kind, tri4[p], tri4[q]);
    for (int c = 0; c < 3; ++c) slot[c] = first ? o.sp[c] : o.sq[c];
    const int A = o.P[0], B = o.P[1], C = o.P[2], D0 = o.Q[0], D1 = o.Q[1], D2 = o.Q[2];
    const double ax = verts[3 * A], ay = verts[3 * A + 1], az = verts[3 * A + 2];
    const double bax = verts[3 * B] - ax, bay = verts[3 * B + 1] - ay, baz = verts[3 * B + 2] - az;
    const double cbx = verts[3 * C] - verts[3 * B], cby = verts[3 * C + 1] - verts[3 * B + 1],
                 cbz = verts[3 * C + 2] - verts[3 * B + 2];
    const double dx0 = verts[3 * D0], dy0 = verts[3 * D0 + 1], dz0 = verts[3 * D0 + 2];
    const double e1x = verts[3 * D1] - dx0, e1y = verts[3 * D1 + 1] - dy0, e1z = verts[3 * D1 + 2] - dz0;
    const double e2x = verts[3 * D2] - verts[3 * D1], e2y = verts[3 * D2 + 1] - verts[3 * D1 + 1],
                 e2z = verts[3 * D2 + 2] - verts[3 * D1 + 2];
    const double ap = area[p], aq = area[q];
    // the order of the canonical pair, as for its matrix entry
    const int n = ss_order_of(ss, kind, cen4[p].w, ap, cen4[q].w, aq);
    ss_points_n(kind, ss, n, lane, [&](double x1, double x2, double y1, double y2, double wgt) {
      const double px = ax + x1 * bax + x2 * cbx, py = ay + x1 * bay + x2 * cby, pz = az + x1 * baz + x2 * cbz;
      const double qx = dx0 + y1 * e1x + y2 * e2x, qy = dy0 + y1 * e1y + y2 * e2y, qz = dz0 + y1 * e1z + y2 * e2z;
      const double rx = px - qx, ry = py - qy, rz = pz - qz;
      const double f = wgt * rsqrt64(rx * rx + ry * ry + rz * rz);
      const double u1 = first ? x1 : y1, u2 = first ? x2 : y2;
      mc0 = __builtin_fma(1.0 - u1, f, mc0);
      mc1 = __builtin_fma(u1 - u2, f, mc1);
      mc2 = __builtin_fma(u2, f, mc2);
    });
    scale = (2.0 * ap) * (2.0 * aq) * kInv4Pi;
  }
  mc0 = wave_sum(mc0) * scale;
  mc1 = wave_sum(mc1) * scale;
  mc2 = wave_sum(mc2) * scale;
  if (lane == 0) {
    // the canonical vertices' moments into T_i's input slots (a permutation)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      tv[3 * e + k] = (slot[0] == k ? mc0 : 0.0) + (slot[1] == k ? mc1 : 0.0) + (slot[2] == k ? mc2 : 0.0);
  }
}

// m_k(T_i) = (2|T_i| / 4pi) sum_c part[c][i][k] + sum_{e in row i} Phi_{col e} tv[e][k],
// both in a fixed order, then mu(T_i)^2 = 36 diam |sum_k m_k e_k|^2 / |T|^3.
__global__ __launch_bounds__(kWG) void k_res_finish(const double *__restrict__ verts, const int4 *__restrict__ tri4,
                                                    const double4 *__restrict__ cen4, const double *__restrict__ area,
                                                    const double *__restrict__ sigma, const double *__restrict__ part,
                                                    int C, const int32_t *__restrict__ prowptr,
                                                    const int32_t *__restrict__ pcol, const double *__restrict__ tv,
                                                    int N, double *__restrict__ mu2, double *__restrict__ mom) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i >= N) return;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  for (int c = 0; c < C; ++c) {
    const double *q = part + ((size_t)c * N + i) * 3;
    f0 += q[0]; f1 += q[1]; f2 += q[2];
  }
  const double Ti = area[i];
  const double sc = 2.0 * Ti * kInv4Pi;
  double m0 = f0 * sc, m1 = f1 * sc, m2 = f2 * sc;
  for (int e = prowptr[i]; e < prowptr[i + 1]; ++e) {
    const double pj = sigma[pcol[e]];
    m0 = __builtin_fma(pj, tv[3 * e], m0);
    m1 = __builtin_fma(pj, tv[3 * e + 1], m1);
    m2 = __builtin_fma(pj, tv[3 * e + 2], m2);
  }
  if (mom) {
    mom[3 * i] = m0; mom[3 * i + 1] = m1; mom[3 * i + 2] = m2;
  }
  const int4 t = tri4[i];
  const double *P0 = verts + 3 * t.x, *P1 = verts + 3 * t.y, *P2 = verts + 3 * t.z;
  // sum_k m_k e_k with e_0 = P2 - P1, e_1 = P0 - P2, e_2 = P1 - P0
  double v[3];
  for (int d = 0; d < 3; ++d) v[d] = m0 * (P2[d] - P1[d]) + m1 * (P0[d] - P2[d]) + m2 * (P1[d] - P0[d]);
  const double diam = sqrt(cen4[i].w);
  mu2[i] = 36.0 * diam * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (Ti * Ti * Ti);
}

size_t residual_workspace_bytes(int64_t N, int64_t nnz) { return ResLayout(N, nnz).total; }

template <int Q>
static void res_far_launch(const MeshView &m, const double *sigma, const ResRule &rr, int N, int C, int chunk,
                           double *part, hipStream_t s) {
  const dim3 grid((unsigned)((N + kWG - 1) / kWG), (unsigned)C);
  hipLaunchKernelGGL(k_res_far<Q>, grid, dim3(kWG), 0, s, m.qpA64, m.tri4, sigma, rr, N, chunk, part);
}

int launch_residual(const double *verts, int64_t N, const bc_assembly_opts &o, const void *mesh_ws,
                    const void *pattern, int64_t nnz, const double *sigma, double *mu2, double *mom, void *ws,
                    hipStream_t s) {
  const MeshView m = mesh_view(mesh_ws, N);
  const ResLayout L(N, nnz);
  char *w = static_cast<char *>(ws);
  double *part = reinterpret_cast<double *>(w + L.part);
  double *tv = reinterpret_cast<double *>(w + L.tv);
  // the far rule's weights times the barycentric coordinates of its points
  const int n = o.far_order;
  double x[8], wq[8];
  gauss_legendre01(n, x, wq);
  ResRule rr{};
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const int k = a * n + b;
      const double ss = x[a], tt = x[b] * (1.0 - x[a]), wk = wq[a] * wq[b] * (1.0 - x[a]);
      rr.wl[0][k] = wk * (1.0 - ss - tt);
      rr.wl[1][k] = wk * ss;
      rr.wl[2][k] = wk * tt;
    }
  const int C = L.C;
  const int chunk = (int)((N + C - 1) / C);
  switch (n) {
    case 1: res_far_launch<1>(m, sigma, rr, (int)N, C, chunk, part, s); break;
    case 2: res_far_launch<4>(m, sigma, rr, (int)N, C, chunk, part, s); break;
    case 3: res_far_launch<9>(m, sigma, rr, (int)N, C, chunk, part, s); break;
    case 4: res_far_launch<16>(m, sigma, rr, (int)N, C, chunk, part, s); break;
    default: return BC_EINVAL;
  }
  if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  PatternLayout P(N, nnz, o.precision);
  const char *pb = static_cast<const char *>(pattern);
  const int32_t *prowptr = reinterpret_cast<const int32_t *>(pb + P.rowptr);
  const int32_t *pcol = reinterpret_cast<const int32_t *>(pb + P.col);
  const int32_t *prow = reinterpret_cast<const int32_t *>(pb + P.row);
  const int32_t *pkind = reinterpret_cast<const int32_t *>(pb + P.kind);
  const SSTable ss = ss_table(o);
  const unsigned grid = (unsigned)((nnz + 3) / 4);
  hipLaunchKernelGGL(k_res_touch, dim3(grid), dim3(kWG), 0, s, verts, m.tri4, m.cen4, m.area, ss, prow, pcol, pkind,
                     nnz, tv);
  if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  hipLaunchKernelGGL(k_res_finish, dim3((unsigned)((N + kWG - 1) / kWG)), dim3(kWG), 0, s, verts, m.tri4, m.cen4,
                     m.area, sigma, (const double *)part, C, prowptr, pcol, (const double *)tv, (int)N, mu2, mom);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
