// Dual-mesh Galerkin system with operator preconditioning (the paper's
// Algorithm 1, step (i); Section 2.6, eq. "laplace_precond_discrete").
//
// The unknowns are the coefficients x_j of the dual-cell indicators
// chi_j^dual, one per vertex of the primal mesh (N triangles, M vertices).
// Everything is expressed through V_bary, the P0 Galerkin matrix of the
// single-layer operator on the barycentric refinement (6N triangles; son
// 6t + s of triangle t lies in the dual cell of its vertex SON_VERTEX[s]):
//
//   V_dual = P^T V_bary P,                    (P x)_k = x_{owner(k)}
//   D      = sum_m Q_m^T V_bary Q_m,          (Q_m x)_k = (curl_G sum_j x_j phi_j)_m on son k
//   D_reg  = D + a a^T,                       a_j = <phi_j, 1>
//   M[i][j] = <phi_j, chi_i^dual>             (11|T|/54 on the diagonal, 7|T|/108 off it, per triangle)
//
// GMRES solves  M^{-1} V_dual M^{-1} D_reg  x~ = M^{-1} f  (M is symmetric),
// and x = M^{-1} D_reg x~ solves V_dual x = f, f_j = |T_j^dual|.  M^{-1} is
// applied as a fixed number of Jacobi sweeps: a fixed linear operator, used
// the same way on both sides, so the solution is exact whatever the sweep
// count; the count only sets the quality of the preconditioner.  Each GMRES
// step applies V_bary to four vectors in two passes over the matrix: the
// three curl components together, then the dual indicator.  V_bary is FP64,
// or FP32 with the FP64 correction of its touching and near entries; the
// vectors and sums are FP64 either way.  Every reduction has a fixed order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bc_internal.h"

namespace bc {

namespace {

// per corner a of a triangle, its two sons (the dual cell of that vertex)
__device__ __forceinline__ void sons_of_corner(int a, int &s1, int &s2) {
  s1 = a == 0 ? 0 : (a == 1 ? 1 : 3);
  s2 = a == 0 ? 5 : (a == 1 ? 2 : 4);
}

// Per triangle: area, diameter and the surface curls of its three hat
// functions, curl_G phi_a = (P_{a+1} - P_{a+2}) / (2 |T|).
__global__ void k_dual_geometry(const double *__restrict__ verts, const int32_t *__restrict__ tris, int N,
                                double *__restrict__ area, double *__restrict__ diam, double *__restrict__ curl) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double P[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) P[a][c] = verts[3 * tris[3 * t + a] + c];
  const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
  const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
  const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double A2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  area[t] = 0.5 * A2;
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    double l2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      curl[9 * t + 3 * a + k] = (P[b][k] - P[c][k]) / A2;
      l2 += (P[b][k] - P[a][k]) * (P[b][k] - P[a][k]);
    }
    d2 = fmax(d2, l2);
  }
  diam[t] = sqrt(d2);
}

// Per vertex: f_j = |T_j^dual| = sum_{T ni j} |T|/3 (also a_j = <phi_j, 1>)
// and the mass matrix diagonal sum_{T ni j} 11|T|/54, in incidence order.
__global__ void k_dual_vertex(const int32_t *__restrict__ iptr, const int32_t *__restrict__ itri, int M,
                              const double *__restrict__ area, double *__restrict__ f, double *__restrict__ mdiag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double s = 0.0;
  for (int e = iptr[j]; e < iptr[j + 1]; ++e) s += area[itri[e]];
  f[j] = s / 3.0;
  mdiag[j] = s * (11.0 / 54.0);
}

// out_k = x_{owner(k)} for the 6N sons
__global__ void k_dual_P(const double *__restrict__ x, const int32_t *__restrict__ tris, int N,
                         double *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 6 * N) return;
  const int t = k / 6, s = k - 6 * t;
  const int sv = s == 0 || s == 5 ? 0 : (s <= 2 ? 1 : 2);  // sons 0, 5 touch v0; 1, 2 touch v1; 3, 4 touch v2
  out[k] = x[tris[3 * t + sv]];
}

// out[m][k] = sum_a curl[t][a][m] x_{tris[t][a]} for the sons k of t
__global__ void k_dual_Q(const double *__restrict__ x, const int32_t *__restrict__ tris,
                         const double *__restrict__ curl, int N, int64_t nb, double *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 6 * N) return;
  const int t = k / 6;
  const double x0 = x[tris[3 * t]], x1 = x[tris[3 * t + 1]], x2 = x[tris[3 * t + 2]];
  for (int m = 0; m < 3; ++m) {
    const double v = curl[9 * t + m] * x0 + curl[9 * t + 3 + m] * x1 + curl[9 * t + 6 + m] * x2;
    out[m * nb + k] = v;
  }
}

// out_j = sum over the triangles around j (incidence order) of the two sons
// in j's dual cell: (P^T y)_j
__global__ void k_dual_PT(const double *__restrict__ y, const int32_t *__restrict__ iptr,
                          const int32_t *__restrict__ itri, const int32_t *__restrict__ icor, int M,
                          double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double s = 0.0;
  for (int e = iptr[j]; e < iptr[j + 1]; ++e) {
    int s1, s2;
    sons_of_corner(icor[e], s1, s2);
    const int t = itri[e];
    s += y[6 * t + s1] + y[6 * t + s2];
  }
  out[j] = s;
}

// out_j = sum_m (Q_m^T y_m)_j + a_j (a^T u), with (a^T u) read from *au
__global__ void k_dual_QT(const double *__restrict__ y, int64_t nb, const int32_t *__restrict__ iptr,
                          const int32_t *__restrict__ itri, const int32_t *__restrict__ icor,
                          const double *__restrict__ curl, const double *__restrict__ a, const double *__restrict__ au,
                          int M, double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double s = 0.0;
  for (int e = iptr[j]; e < iptr[j + 1]; ++e) {
    const int t = itri[e], c = icor[e];
    for (int m = 0; m < 3; ++m) {
      const double *ym = y + m * nb + 6 * t;
      const double sum6 = ((ym[0] + ym[1]) + (ym[2] + ym[3])) + (ym[4] + ym[5]);
      s = fma(curl[9 * t + 3 * c + m], sum6, s);
    }
  }
  out[j] = fma(a[j], *au, s);
}

// One Jacobi sweep for M z = r: zout = zin + (r - M zin) / diag(M), with
// (M z)_i = sum_{T ni i} |T| (11/54 z_i + 7/108 (z_b + z_c)).
__global__ void k_dual_jacobi(const double *__restrict__ r, const double *__restrict__ zin,
                              const int32_t *__restrict__ iptr, const int32_t *__restrict__ itri,
                              const int32_t *__restrict__ icor, const int32_t *__restrict__ tris,
                              const double *__restrict__ area, const double *__restrict__ mdiag, int M,
                              double *__restrict__ zout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double zi = zin[i];
  double mz = 0.0;
  for (int e = iptr[i]; e < iptr[i + 1]; ++e) {
    const int t = itri[e], c = icor[e];
    const double zb = zin[tris[3 * t + (c + 1) % 3]], zc = zin[tris[3 * t + (c + 2) % 3]];
    mz = fma(area[t], (11.0 / 54.0) * zi + (7.0 / 108.0) * (zb + zc), mz);
  }
  zout[i] = zi + (r[i] - mz) / mdiag[i];
}

__global__ void k_dual_div(const double *__restrict__ r, const double *__restrict__ d, int M, double *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) z[i] = r[i] / d[i];
}

// out[q] = sum_i A[q][i] w_i for q < nq (rows of A at stride lda): one
// workgroup per q, fixed order (strided per thread, then a tree in LDS).
__global__ __launch_bounds__(kWG) void k_multidot(const double *__restrict__ A, int64_t lda, const double *__restrict__ w,
                                                  int M, double *__restrict__ out) {
  __shared__ double part[kWG];
  const int q = blockIdx.x;
  const double *aq = A + q * lda;
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += kWG) s = fma(aq[i], w[i], s);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = part[0];
}

// w_i -= sum_{q < nq} h_q A[q][i] (q ascending)
__global__ void k_gs_update(const double *__restrict__ A, int64_t lda, const double *__restrict__ h, int nq, int M,
                            double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double s = w[i];
  for (int q = 0; q < nq; ++q) s = fma(-h[q], A[q * lda + i], s);
  w[i] = s;
}

// y_m[i] += sum_e corr[e] x_m[col[e]] over row i of the pattern (e
// ascending), for the NR vectors at stride n: the FP64 correction of the
// touching and near entries of an FP32 matrix.
template <int NR>
__global__ void k_csr_add(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          const double *__restrict__ corr, int n, int64_t stride, const double *__restrict__ x,
                          double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc[NR];
  for (int m = 0; m < NR; ++m) acc[m] = y[m * stride + i];
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const double c = corr[e];
    const int j = col[e];
    for (int m = 0; m < NR; ++m) acc[m] = fma(c, x[m * stride + j], acc[m]);
  }
  for (int m = 0; m < NR; ++m) y[m * stride + i] = acc[m];
}

// out_i = v
__global__ void k_fill(double v, int n, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

// out_i = alpha * in_i
__global__ void k_scale(const double *__restrict__ in, double alpha, int M, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) out[i] = alpha * in[i];
}

// out_i = sum_q c_q A[q][i] (q ascending)
__global__ void k_combine(const double *__restrict__ A, int64_t lda, const double *__restrict__ c, int nq, int M,
                          double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double s = 0.0;
  for (int q = 0; q < nq; ++q) s = fma(c[q], A[q * lda + i], s);
  out[i] = s;
}

// eta_T^2 = h_T || Phi - I Phi ||^2_{L2(T)} (eq. "zz:T"): on each son the
// difference is affine with values g at the son's vertices, and
// int g^2 = |son| / 12 ((sum g)^2 + sum g^2).  Son (v_a, m_ab, c) of the
// cell of a: g = (0, (x_a - x_b)/2, x_a - mean); son (m_ca, v_a, c):
// g = ((x_a - x_c)/2, 0, x_a - mean); |son| = |T| / 6.
__global__ void k_dual_zz(const double *__restrict__ x, const int32_t *__restrict__ tris,
                          const double *__restrict__ area, const double *__restrict__ diam, int N, int h_mode,
                          double *__restrict__ eta2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double v[3] = {x[tris[3 * t]], x[tris[3 * t + 1]], x[tris[3 * t + 2]]};
  const double mean = (v[0] + v[1] + v[2]) / 3.0;
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double gc = v[a] - mean;
    const double g1 = 0.5 * (v[a] - v[b]), g2 = 0.5 * (v[a] - v[c]);
    // son towards b: (0, g1, gc); son towards c: (g2, 0, gc)
    const double s1 = g1 + gc, s2 = g2 + gc;
    s += (s1 * s1 + g1 * g1 + gc * gc) + (s2 * s2 + g2 * g2 + gc * gc);
  }
  const double h = h_mode == 0 ? diam[t] : sqrt(area[t]);
  eta2[t] = h * (area[t] / 6.0) / 12.0 * s;
}

inline int blocks(int64_t n) { return (int)((n + kWG - 1) / kWG); }

}  // namespace

// ---------------------------------------------------------------- layout
// dots: [0, restart) Gram-Schmidt inner products and norms; restart + 4:
// a^T u of D_reg; [restart + 8, 2 restart + 8): a row of the energy Gram
// matrix; 2 restart + 8: sum of eta^2; [2 restart + 9, 3 restart + 9): the
// coefficients y of the current iterate.
constexpr int64_t kDotsAu = 4, kDotsGram = 8;
DualLayout::DualLayout(int64_t N, int64_t M, int32_t restart) {
  nb = 6 * N;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = (o + bytes + 255) & ~size_t(255);
    return r;
  };
  area = take(8 * N);
  diam = take(8 * N);
  curl = take(8 * 9 * N);
  f = take(8 * M);
  mdiag = take(8 * M);
  basis = take(8 * (size_t)(restart + 1) * M);
  wbas = take(8 * (size_t)restart * M);  // M^{-1} D_reg z_i
  ubas = take(8 * (size_t)restart * M);  // V_dual M^{-1} D_reg z_i
  w = take(8 * M);
  t1 = take(8 * M);
  t2 = take(8 * M);
  t3 = take(8 * M);
  eta2 = take(8 * N);
  ones = take(8 * N);
  bvec = take(8 * 4 * (size_t)nb);  // three curl components and the dual indicator
  yvec = take(8 * 4 * (size_t)nb);
  dots = take(8 * (size_t)(3 * restart + 16));
  size_t mvb = 0;  // the largest product scratch of the FP64 and the FP32-matrix kinds
  for (int32_t kind : {(int32_t)BC_FP64, kMatvecF32X64})
    for (int nr : {1, 3}) mvb = std::max(mvb, MatvecLayout(nb, kind, nr).total);
  mv = take(mvb);
  total = o;
}

int launch_dual_setup(const double *verts, const int32_t *tris, int64_t N, int64_t M, const int32_t *iptr,
                      const int32_t *itri, void *ws, int32_t restart, hipStream_t s) {
  const DualLayout L(N, M, restart);
  char *b = static_cast<char *>(ws);
  double *area = reinterpret_cast<double *>(b + L.area), *diam = reinterpret_cast<double *>(b + L.diam);
  hipLaunchKernelGGL(k_dual_geometry, dim3(blocks(N)), dim3(kWG), 0, s, verts, tris, (int)N, area, diam,
                     reinterpret_cast<double *>(b + L.curl));
  hipLaunchKernelGGL(k_dual_vertex, dim3(blocks(M)), dim3(kWG), 0, s, iptr, itri, (int)M, (const double *)area,
                     reinterpret_cast<double *>(b + L.f), reinterpret_cast<double *>(b + L.mdiag));
  hipLaunchKernelGGL(k_fill, dim3(blocks(N)), dim3(kWG), 0, s, 1.0, (int)N, reinterpret_cast<double *>(b + L.ones));
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

// y = R^{-1} g for the leading n x n upper triangle of the rotated Hessenberg
// matrix (row stride m).
static void back_substitute(const std::vector<double> &H, int m, const std::vector<double> &g, int n,
                            std::vector<double> &y) {
  y.assign(n, 0.0);
  for (int q = n - 1; q >= 0; --q) {
    double sum = g[q];
    for (int c = q + 1; c < n; ++c) sum -= H[(size_t)q * m + c] * y[c];
    y[q] = sum / H[(size_t)q * m + q];
  }
}

// Host-driven GMRES (no restart within max_iter <= restart): Arnoldi with
// classical Gram-Schmidt applied twice (all inner products of a pass in one
// launch), Givens rotations on the host.  Besides the Krylov basis z_i it
// keeps w_i = M^{-1} D_reg z_i and u_i = V_dual w_i, which the operator forms
// anyway: the iterate is x_k = sum_i y_i w_i without a further product, and
// the energy norm of an update x_k - x_{k-1} = sum_i dy_i w_i is
// dy^T G dy with G_ij = w_i^T u_j, one new row of inner products per step.
int run_dual_solve(const void *Vb, int32_t precision, const void *pattern, int64_t nnz, const int32_t *tris, int64_t N,
                   int64_t M, const int32_t *iptr, const int32_t *itri, const int32_t *icor, void *ws,
                   const bc_dual_opts &o, double *x, bc_dual_result *res, hipStream_t s) {
  const DualLayout L(N, M, o.restart);
  const bool mixed = precision == BC_MIXED;
  const int32_t kind = mixed ? kMatvecF32X64 : (int32_t)BC_FP64;
  const PatternLayout PL(6 * N, nnz, BC_MIXED);
  const char *pb = static_cast<const char *>(pattern);
  const int32_t *prow = mixed ? reinterpret_cast<const int32_t *>(pb + PL.rowptr) : nullptr;
  const int32_t *pcol = mixed ? reinterpret_cast<const int32_t *>(pb + PL.col) : nullptr;
  const double *pcorr = mixed ? reinterpret_cast<const double *>(pb + PL.corr) : nullptr;
  char *b = static_cast<char *>(ws);
  auto D = [&](size_t off) { return reinterpret_cast<double *>(b + off); };
  const double *area = D(L.area), *diam = D(L.diam), *curl = D(L.curl), *f = D(L.f), *mdiag = D(L.mdiag);
  double *basis = D(L.basis), *wbas = D(L.wbas), *ubas = D(L.ubas), *w = D(L.w), *t1 = D(L.t1), *t2 = D(L.t2),
         *t3 = D(L.t3), *eta2 = D(L.eta2);
  const double *ones = D(L.ones);
  double *bvec = D(L.bvec), *yvec = D(L.yvec), *dots = D(L.dots);
  double *dots_au = dots + o.restart + kDotsAu, *dots_gram = dots + o.restart + kDotsGram;
  double *dots_eta = dots + 2 * o.restart + kDotsGram, *dots_y = dots + 2 * o.restart + kDotsGram + 1;
  void *mvws = b + L.mv;
  const int64_t nb = L.nb;
  const int gM = blocks(M), gB = blocks(nb), gN = blocks(N);
  const bool inexact = o.inexact_lambda > 0.0;
  bool err = false;
  auto chk = [&]() { err = err || hipGetLastError() != hipSuccess; };
  // z = M^{-1} r by o.jacobi_sweeps Jacobi sweeps from z0 = r / diag (ping-pong t2/t3)
  auto minv = [&](const double *r, double *z) {
    hipLaunchKernelGGL(k_dual_div, dim3(gM), dim3(kWG), 0, s, r, mdiag, (int)M, t2);
    double *cur = t2, *nxt = t3;
    for (int k = 0; k < o.jacobi_sweeps; ++k) {
      hipLaunchKernelGGL(k_dual_jacobi, dim3(gM), dim3(kWG), 0, s, r, (const double *)cur, iptr, itri, icor, tris,
                         area, mdiag, (int)M, nxt);
      double *tmp = cur; cur = nxt; nxt = tmp;
    }
    hipLaunchKernelGGL(k_scale, dim3(gM), dim3(kWG), 0, s, (const double *)cur, 1.0, (int)M, z);
    chk();
  };
  // out = D_reg u: the three curl components share one pass over V_bary
  auto dreg = [&](const double *u, double *out) {
    hipLaunchKernelGGL(k_dual_Q, dim3(gB), dim3(kWG), 0, s, u, tris, curl, (int)N, nb, bvec);
    if (launch_matvec(kind, Vb, nb, 3, bvec, yvec, mvws, s) != BC_OK) err = true;
    if (mixed)
      hipLaunchKernelGGL(k_csr_add<3>, dim3(gB), dim3(kWG), 0, s, prow, pcol, pcorr, (int)nb, nb,
                         (const double *)bvec, yvec);
    hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, f, (int64_t)0, u, (int)M, dots_au);
    hipLaunchKernelGGL(k_dual_QT, dim3(gM), dim3(kWG), 0, s, (const double *)yvec, nb, iptr, itri, icor, curl, f,
                       (const double *)dots_au, (int)M, out);
    chk();
  };
  // out = V_dual u = P^T V_bary P u
  auto vdual = [&](const double *u, double *out) {
    hipLaunchKernelGGL(k_dual_P, dim3(gB), dim3(kWG), 0, s, u, tris, (int)N, bvec + 3 * nb);
    if (launch_matvec(kind, Vb, nb, 1, bvec + 3 * nb, yvec + 3 * nb, mvws, s) != BC_OK) err = true;
    if (mixed)
      hipLaunchKernelGGL(k_csr_add<1>, dim3(gB), dim3(kWG), 0, s, prow, pcol, pcorr, (int)nb, nb,
                         (const double *)(bvec + 3 * nb), yvec + 3 * nb);
    hipLaunchKernelGGL(k_dual_PT, dim3(gM), dim3(kWG), 0, s, (const double *)(yvec + 3 * nb), iptr, itri, icor,
                       (int)M, out);
    chk();
  };
  // asynchronous reads of device values; wait() makes them valid
  auto read = [&](const double *src, int n, std::vector<double> &h) {
    h.resize(n);
    if (hipMemcpyAsync(h.data(), src, 8 * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess) err = true;
  };
  auto wait = [&]() {
    if (hipStreamSynchronize(s) != hipSuccess) err = true;
  };
  const int m = o.max_iter;
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0), h, hg, he, G((size_t)m * m, 0.0);
  std::vector<double> y, yprev;
  // rhs = M^{-1} f, v0 = rhs / |rhs|
  minv(f, w);
  hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, (const double *)w, (int64_t)0, (const double *)w, (int)M, dots);
  read(dots, 1, h);
  wait();
  if (err) return BC_EDEVICE;
  const double beta = sqrt(h[0]);
  if (!(beta > 0.0)) return BC_EINVAL;
  hipLaunchKernelGGL(k_scale, dim3(gM), dim3(kWG), 0, s, (const double *)w, 1.0 / beta, (int)M, basis);
  g[0] = beta;
  int k = 0;
  double rel = 1.0, energy = 0.0, eta = 0.0;
  int status = BC_ENOCONV, stop = 0;
  for (; k < m; ++k) {
    const double *vk = basis + (size_t)k * M;
    double *wk = wbas + (size_t)k * M, *uk = ubas + (size_t)k * M;
    // w_k = M^{-1} D_reg z_k, u_k = V_dual w_k, Arnoldi vector M^{-1} u_k
    dreg(vk, t1);
    minv(t1, wk);
    vdual(wk, uk);
    minv(uk, w);
    if (inexact) {
      hipLaunchKernelGGL(k_multidot, dim3(k + 1), dim3(kWG), 0, s, (const double *)ubas, (int64_t)M,
                         (const double *)wk, (int)M, dots_gram);
      read(dots_gram, k + 1, hg);
    }
    // two passes of classical Gram-Schmidt against v_0 .. v_k
    std::vector<double> hk(k + 2, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_multidot, dim3(k + 1), dim3(kWG), 0, s, (const double *)basis, (int64_t)M,
                         (const double *)w, (int)M, dots);
      hipLaunchKernelGGL(k_gs_update, dim3(gM), dim3(kWG), 0, s, (const double *)basis, (int64_t)M,
                         (const double *)dots, k + 1, (int)M, w);
      read(dots, k + 1, h);
      wait();
      for (int q = 0; q <= k; ++q) hk[q] += h[q];
    }
    hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, (const double *)w, (int64_t)0, (const double *)w, (int)M,
                       dots);
    read(dots, 1, h);
    wait();
    if (err) return BC_EDEVICE;
    if (inexact)
      for (int q = 0; q <= k; ++q) G[(size_t)k * m + q] = G[(size_t)q * m + k] = hg[q];
    hk[k + 1] = sqrt(h[0]);
    // previous rotations, then a new one that zeroes hk[k+1]
    for (int q = 0; q < k; ++q) {
      const double a = hk[q], bq = hk[q + 1];
      hk[q] = cs[q] * a + sn[q] * bq;
      hk[q + 1] = -sn[q] * a + cs[q] * bq;
    }
    const double r = std::hypot(hk[k], hk[k + 1]);
    cs[k] = r > 0.0 ? hk[k] / r : 1.0;
    sn[k] = r > 0.0 ? hk[k + 1] / r : 0.0;
    const double hn = hk[k + 1];
    hk[k] = r;
    hk[k + 1] = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    for (int q = 0; q <= k; ++q) H[(size_t)q * m + k] = hk[q];
    rel = fabs(g[k + 1]) / beta;
    if (rel <= o.rtol) stop = 1;
    else if (!(hn > 0.0)) stop = 3;  // exact invariant subspace
    if (inexact) {
      // x_k and its update's energy norm; eta(x_k) from the ZZ indicators
      back_substitute(H, m, g, k + 1, y);
      double e2 = 0.0;
      for (int i = 0; i <= k; ++i) {
        const double di = y[i] - (i < (int)yprev.size() ? yprev[i] : 0.0);
        for (int j = 0; j <= k; ++j) e2 += di * G[(size_t)i * m + j] * (y[j] - (j < (int)yprev.size() ? yprev[j] : 0.0));
      }
      if (hipMemcpyAsync(dots_y, y.data(), 8 * (size_t)(k + 1), hipMemcpyHostToDevice, s) != hipSuccess) err = true;
      hipLaunchKernelGGL(k_combine, dim3(gM), dim3(kWG), 0, s, (const double *)wbas, (int64_t)M,
                         (const double *)dots_y, k + 1, (int)M, x);
      hipLaunchKernelGGL(k_dual_zz, dim3(gN), dim3(kWG), 0, s, (const double *)x, tris, area, diam, (int)N, o.h_mode,
                         eta2);
      hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, (const double *)eta2, (int64_t)0, ones, (int)N,
                         dots_eta);
      read(dots_eta, 1, he);
      wait();
      chk();
      if (err) return BC_EDEVICE;
      energy = sqrt(e2 > 0.0 ? e2 : 0.0);
      eta = sqrt(he[0] > 0.0 ? he[0] : 0.0);
      yprev = y;
      if (stop == 0 && energy <= o.inexact_lambda * eta) stop = 2;
    }
    if (stop != 0) {
      status = BC_OK;
      ++k;
      break;
    }
    if (k + 1 < m) hipLaunchKernelGGL(k_scale, dim3(gM), dim3(kWG), 0, s, (const double *)w, 1.0 / hn, (int)M,
                                      basis + (size_t)(k + 1) * M);
  }
  // x = sum_i y_i w_i with y = R^{-1} g (k x k)
  back_substitute(H, m, g, k, y);
  if (hipMemcpyAsync(dots_y, y.data(), 8 * (size_t)k, hipMemcpyHostToDevice, s) != hipSuccess) err = true;
  hipLaunchKernelGGL(k_combine, dim3(gM), dim3(kWG), 0, s, (const double *)wbas, (int64_t)M, (const double *)dots_y, k,
                     (int)M, x);
  // Cap = (1/4pi) f^T x
  hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, f, (int64_t)0, (const double *)x, (int)M, dots);
  read(dots, 1, h);
  wait();
  chk();
  if (err) return BC_EDEVICE;
  res->cap = h[0] * kInv4Pi;
  res->rel_residual = rel;
  res->energy_step = inexact ? energy : 0.0;
  res->eta = inexact ? eta : 0.0;
  res->iters = k;
  res->status = status;
  res->stop = stop;
  res->reserved = 0;
  return BC_OK;
}

int launch_dual_zz(const void *ws, const int32_t *tris, int64_t N, int64_t M, int32_t restart, const double *x,
                   int h_mode, double *eta2, hipStream_t s) {
  const DualLayout L(N, M, restart);
  const char *b = static_cast<const char *>(ws);
  hipLaunchKernelGGL(k_dual_zz, dim3(blocks(N)), dim3(kWG), 0, s, x, tris, reinterpret_cast<const double *>(b + L.area),
                     reinterpret_cast<const double *>(b + L.diam), (int)N, h_mode, eta2);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
