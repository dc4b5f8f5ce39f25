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
__global__ void k_dual_P(const int32_t *__restrict__ skip, const double *__restrict__ x,
                         const int32_t *__restrict__ tris, int N, double *__restrict__ out) {
  if (*skip) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 6 * N) return;
  const int t = k / 6, s = k - 6 * t;
  const int sv = s == 0 || s == 5 ? 0 : (s <= 2 ? 1 : 2);  // sons 0, 5 touch v0; 1, 2 touch v1; 3, 4 touch v2
  out[k] = x[tris[3 * t + sv]];
}

// out[m][k] = sum_a curl[t][a][m] x_{tris[t][a]} for the sons k of t
__global__ void k_dual_Q(const int32_t *__restrict__ skip, const double *__restrict__ x,
                         const int32_t *__restrict__ tris, const double *__restrict__ curl, int N, int64_t nb,
                         double *__restrict__ out) {
  if (*skip) return;
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
__global__ void k_dual_PT(const int32_t *__restrict__ skip, const double *__restrict__ y,
                          const int32_t *__restrict__ iptr, const int32_t *__restrict__ itri,
                          const int32_t *__restrict__ icor, int M, double *__restrict__ out) {
  if (*skip) return;
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
__global__ void k_dual_QT(const int32_t *__restrict__ skip, const double *__restrict__ y, int64_t nb,
                          const int32_t *__restrict__ iptr, const int32_t *__restrict__ itri,
                          const int32_t *__restrict__ icor, const double *__restrict__ curl,
                          const double *__restrict__ a, const double *__restrict__ au, int M,
                          double *__restrict__ out) {
  if (*skip) return;
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
__global__ void k_dual_jacobi(const int32_t *__restrict__ skip, const double *__restrict__ r,
                              const double *__restrict__ zin, const int32_t *__restrict__ iptr,
                              const int32_t *__restrict__ itri, const int32_t *__restrict__ icor,
                              const int32_t *__restrict__ tris, const double *__restrict__ area,
                              const double *__restrict__ mdiag, int M, double *__restrict__ zout) {
  if (*skip) return;
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

__global__ void k_dual_div(const int32_t *__restrict__ skip, const double *__restrict__ r,
                           const double *__restrict__ d, int M, double *__restrict__ z) {
  if (*skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) z[i] = r[i] / d[i];
}

// out[q] = sum_i A[q][i] w_i for q < nq (rows of A at stride lda): one
// workgroup per q, fixed order (strided per thread, then a tree in LDS).
__global__ __launch_bounds__(kWG) void k_multidot(const int32_t *__restrict__ skip, const double *__restrict__ A,
                                                  int64_t lda, const double *__restrict__ w, int M,
                                                  double *__restrict__ out) {
  if (*skip) return;
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
__global__ void k_gs_update(const int32_t *__restrict__ skip, const double *__restrict__ A, int64_t lda,
                            const double *__restrict__ h, int nq, int M, double *__restrict__ w) {
  if (*skip) return;
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
__global__ void k_csr_add(const int32_t *__restrict__ skip, const int32_t *__restrict__ rowptr,
                          const int32_t *__restrict__ col, const double *__restrict__ corr, int n, int64_t stride,
                          const double *__restrict__ x, double *__restrict__ y) {
  if (*skip) return;
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

// out_i = alpha * in_i, alpha read from the device
__global__ void k_scale(const int32_t *__restrict__ skip, const double *__restrict__ in,
                        const double *__restrict__ alpha, int M, double *__restrict__ out) {
  if (*skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) out[i] = *alpha * in[i];
}

// out_i = sum_q c_q A[q][i] (q ascending) for q < *nq (device count) or
// q < nq_fixed when nq is NULL
__global__ void k_combine(const int32_t *__restrict__ skip, const double *__restrict__ A, int64_t lda,
                          const double *__restrict__ c, const int32_t *__restrict__ nq, int nq_fixed, int M,
                          double *__restrict__ out) {
  if (*skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int n = nq ? *nq : nq_fixed;
  double s = 0.0;
  for (int q = 0; q < n; ++q) s = fma(c[q], A[q * lda + i], s);
  out[i] = s;
}

// eta_T^2 = h_T || Phi - I Phi ||^2_{L2(T)} (eq. "zz:T"): on each son the
// difference is affine with values g at the son's vertices, and
// int g^2 = |son| / 12 ((sum g)^2 + sum g^2).  Son (v_a, m_ab, c) of the
// cell of a: g = (0, (x_a - x_b)/2, x_a - mean); son (m_ca, v_a, c):
// g = ((x_a - x_c)/2, 0, x_a - mean); |son| = |T| / 6.
__global__ void k_dual_zz(const int32_t *__restrict__ skip, const double *__restrict__ x,
                          const int32_t *__restrict__ tris, const double *__restrict__ area,
                          const double *__restrict__ diam, int N, int h_mode, double *__restrict__ eta2) {
  if (skip && *skip) return;
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

// GMRES control on the device: the scalars of the Arnoldi process and the
// stop decision, written by single-thread kernels, read by the host once per
// batch of steps.  Every kernel of a step skips itself once `done` is set.
struct GCtl {
  int32_t done;   // a stop criterion holds (or the right-hand side vanished)
  int32_t stop;   // 1 residual, 2 inexact-solve criterion, 3 invariant subspace
  int32_t bad;    // zero right-hand side
  int32_t k;      // GMRES steps taken when done
  double beta, rel, hn_inv, energy, eta;
};

// hacc[q] = dots[q] (pass 0) or hacc[q] + dots[q] (pass 1), q < n: the two
// Gram-Schmidt passes' coefficients of one Arnoldi column
__global__ void k_gs_acc(const int32_t *__restrict__ skip, const double *__restrict__ dots, int n, int add,
                         double *__restrict__ hacc) {
  if (*skip) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) hacc[q] = add ? hacc[q] + dots[q] : dots[q];
}

// a cleared control block (no stop yet) and the never-set flag nsteps[1]
__global__ void k_gmres_clear(GCtl *__restrict__ c, int32_t *__restrict__ nsteps) {
  if (threadIdx.x != 0) return;
  c->done = 0; c->stop = 0; c->bad = 0; c->k = 0;
  nsteps[0] = 0;
  nsteps[1] = 0;
}

// beta = |M^{-1} f|; the first basis vector is scaled by 1/beta
__global__ void k_gmres_init(GCtl *__restrict__ c, const double *__restrict__ nrm2, double *__restrict__ g,
                             double *__restrict__ yprev, int m) {
  if (threadIdx.x != 0) return;
  const double beta = sqrt(*nrm2);
  c->done = 0; c->stop = 0; c->bad = 0; c->k = 0;
  c->beta = beta; c->rel = 1.0; c->energy = 0.0; c->eta = 0.0;
  c->hn_inv = beta > 0.0 ? 1.0 / beta : 0.0;
  if (!(beta > 0.0)) { c->bad = 1; c->done = 1; }
  g[0] = beta;
  for (int q = 0; q < m; ++q) yprev[q] = 0.0;
}

// y = R^{-1} g for the leading n x n upper triangle of H (row stride m)
__device__ void back_substitute_dev(const double *H, int m, const double *g, int n, double *y) {
  for (int q = n - 1; q >= 0; --q) {
    double sum = g[q];
    for (int c = q + 1; c < n; ++c) sum -= H[(size_t)q * m + c] * y[c];
    y[q] = sum / H[(size_t)q * m + q];
  }
}

// Step k's Arnoldi column h_0..h_k (hacc) and h_{k+1} = |w| (from *nrm2):
// the previous Givens rotations, a new one zeroing h_{k+1}, the rotated
// right-hand side g and the relative residual |g_{k+1}| / beta; the stop
// decision (residual tolerance, or an exact invariant subspace); 1 / h_{k+1}
// for the next basis vector.  With the inexact stop, also the iterate's
// coefficients y = R^{-1} g (to *ydev) and the energy norm of its update,
// (y - y_prev)^T G (y - y_prev) with G_ij = w_i^T V_dual w_j, whose row k is
// `gram`; the decision then waits for the estimator (k_gmres_inexact).
__global__ void k_gmres_rot(GCtl *__restrict__ c, const double *__restrict__ hacc, const double *__restrict__ nrm2,
                            double *__restrict__ H, double *__restrict__ cs, double *__restrict__ sn,
                            double *__restrict__ g, int k, int m, double rtol, int inexact,
                            const double *__restrict__ gram, double *__restrict__ G, double *__restrict__ y,
                            double *__restrict__ yprev) {
  if (threadIdx.x != 0 || c->done) return;
  double *col = H + k;  // H[q][k] = col[q * m]
  for (int q = 0; q <= k; ++q) col[(size_t)q * m] = hacc[q];
  const double hk1 = sqrt(*nrm2);
  for (int q = 0; q < k; ++q) {
    const double a = col[(size_t)q * m], b = col[(size_t)(q + 1) * m];
    col[(size_t)q * m] = cs[q] * a + sn[q] * b;
    col[(size_t)(q + 1) * m] = -sn[q] * a + cs[q] * b;
  }
  const double hkk = col[(size_t)k * m];
  const double r = hypot(hkk, hk1);
  cs[k] = r > 0.0 ? hkk / r : 1.0;
  sn[k] = r > 0.0 ? hk1 / r : 0.0;
  col[(size_t)k * m] = r;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  const double rel = fabs(g[k + 1]) / c->beta;
  c->rel = rel;
  int stop = 0;
  if (rel <= rtol) stop = 1;
  else if (!(hk1 > 0.0)) stop = 3;  // exact invariant subspace
  c->hn_inv = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
  c->stop = stop;
  if (inexact) {
    for (int q = 0; q <= k; ++q) G[(size_t)k * m + q] = G[(size_t)q * m + k] = gram[q];
    back_substitute_dev(H, m, g, k + 1, y);
    double e2 = 0.0;
    for (int i = 0; i <= k; ++i) {
      const double di = y[i] - yprev[i];
      for (int j = 0; j <= k; ++j) e2 += di * G[(size_t)i * m + j] * (y[j] - yprev[j]);
    }
    for (int i = 0; i <= k; ++i) yprev[i] = y[i];
    c->energy = sqrt(e2 > 0.0 ? e2 : 0.0);
  } else if (stop) {
    c->done = 1;
    c->k = k + 1;
  }
}

// inexact stop (Section 2.5, Remark (i)): eta(x_k) from the summed ZZ
// indicators of the iterate; stop once ||x_k - x_{k-1}||_V <= lambda eta
__global__ void k_gmres_inexact(GCtl *__restrict__ c, const double *__restrict__ eta2_sum, double lambda, int k) {
  if (threadIdx.x != 0 || c->done) return;
  const double e = *eta2_sum;
  c->eta = sqrt(e > 0.0 ? e : 0.0);
  if (c->stop == 0 && c->energy <= lambda * c->eta) c->stop = 2;
  if (c->stop != 0) {
    c->done = 1;
    c->k = k + 1;
  }
}

// the steps taken (max_iter when no criterion held) and their coefficients
// y (H with row stride m)
__global__ void k_gmres_final(GCtl *__restrict__ c, const double *__restrict__ H, const double *__restrict__ g, int m,
                              int max_iter, double *__restrict__ y, int32_t *__restrict__ nsteps) {
  if (threadIdx.x != 0) return;
  const int n = c->bad ? 0 : (c->done ? c->k : max_iter);
  *nsteps = n;
  back_substitute_dev(H, m, g, n, y);
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
  gctl = take(256);                                 // GCtl and the step count
  H = take(8 * (size_t)restart * (size_t)restart);  // rotated Hessenberg matrix (upper triangle)
  G = take(8 * (size_t)restart * (size_t)restart);  // energy Gram matrix (inexact stop)
  rot = take(8 * (size_t)(6 * restart + 8));        // cs, sn, g, y, yprev, hacc
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

constexpr int kGmresBatch = 4;  // GMRES steps queued between two reads of the device's stop decision

// GMRES (no restart within max_iter <= restart): Arnoldi with classical
// Gram-Schmidt applied twice (all inner products of a pass in one launch),
// Givens rotations and the stop decision in single-thread kernels on the
// device.  The host queues kGmresBatch steps at a time and reads the
// device's decision once per batch; steps queued past the stop skip
// themselves.  Besides the Krylov basis z_i it keeps w_i = M^{-1} D_reg z_i
// and u_i = V_dual w_i, which the operator forms anyway: the iterate is
// x_k = sum_i y_i w_i without a further product, and the energy norm of an
// update x_k - x_{k-1} = sum_i dy_i w_i is dy^T G dy with G_ij = w_i^T u_j,
// one new row of inner products per step.
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
  GCtl *ctl = reinterpret_cast<GCtl *>(b + L.gctl);
  int32_t *nsteps = reinterpret_cast<int32_t *>(b + L.gctl + 128);
  const int32_t *skip = &ctl->done;
  double *H = D(L.H), *G = D(L.G), *rot = D(L.rot);
  const int m = o.max_iter, rs = o.restart;
  double *cs = rot, *sn = rot + rs, *g = rot + 2 * rs, *yv = rot + 3 * rs + 1, *yprev = rot + 4 * rs + 1,
         *hacc = rot + 5 * rs + 1;
  void *mvws = b + L.mv;
  const int64_t nb = L.nb;
  const int gM = blocks(M), gB = blocks(nb), gN = blocks(N);
  const bool inexact = o.inexact_lambda > 0.0;
  bool err = false;
  auto chk = [&]() { err = err || hipGetLastError() != hipSuccess; };
  // z = M^{-1} r by o.jacobi_sweeps Jacobi sweeps from z0 = r / diag (ping-pong t2/t3)
  auto minv = [&](const double *r, double *z) {
    hipLaunchKernelGGL(k_dual_div, dim3(gM), dim3(kWG), 0, s, skip, r, mdiag, (int)M, t2);
    double *cur = t2, *nxt = t3;
    for (int k = 0; k < o.jacobi_sweeps; ++k) {
      hipLaunchKernelGGL(k_dual_jacobi, dim3(gM), dim3(kWG), 0, s, skip, r, (const double *)cur, iptr, itri, icor,
                         tris, area, mdiag, (int)M, nxt);
      double *tmp = cur; cur = nxt; nxt = tmp;
    }
    hipLaunchKernelGGL(k_combine, dim3(gM), dim3(kWG), 0, s, skip, (const double *)cur, (int64_t)0, ones,
                       (const int32_t *)nullptr, 1, (int)M, z);  // z = 1 * cur
    chk();
  };
  // out = D_reg u: the three curl components share one pass over V_bary
  auto dreg = [&](const double *u, double *out) {
    hipLaunchKernelGGL(k_dual_Q, dim3(gB), dim3(kWG), 0, s, skip, u, tris, curl, (int)N, nb, bvec);
    if (launch_matvec(kind, Vb, nb, 3, bvec, yvec, mvws, s, skip) != BC_OK) err = true;
    if (mixed)
      hipLaunchKernelGGL(k_csr_add<3>, dim3(gB), dim3(kWG), 0, s, skip, prow, pcol, pcorr, (int)nb, nb,
                         (const double *)bvec, yvec);
    hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, skip, f, (int64_t)0, u, (int)M, dots_au);
    hipLaunchKernelGGL(k_dual_QT, dim3(gM), dim3(kWG), 0, s, skip, (const double *)yvec, nb, iptr, itri, icor, curl, f,
                       (const double *)dots_au, (int)M, out);
    chk();
  };
  // out = V_dual u = P^T V_bary P u
  auto vdual = [&](const double *u, double *out) {
    hipLaunchKernelGGL(k_dual_P, dim3(gB), dim3(kWG), 0, s, skip, u, tris, (int)N, bvec + 3 * nb);
    if (launch_matvec(kind, Vb, nb, 1, bvec + 3 * nb, yvec + 3 * nb, mvws, s, skip) != BC_OK) err = true;
    if (mixed)
      hipLaunchKernelGGL(k_csr_add<1>, dim3(gB), dim3(kWG), 0, s, skip, prow, pcol, pcorr, (int)nb, nb,
                         (const double *)(bvec + 3 * nb), yvec + 3 * nb);
    hipLaunchKernelGGL(k_dual_PT, dim3(gM), dim3(kWG), 0, s, skip, (const double *)(yvec + 3 * nb), iptr, itri,
                       icor, (int)M, out);
    chk();
  };
  // rhs = M^{-1} f, v0 = rhs / |rhs|; the control block starts cleared
  hipLaunchKernelGGL(k_gmres_clear, dim3(1), dim3(64), 0, s, ctl, nsteps);
  minv(f, w);
  hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, skip, (const double *)w, (int64_t)0, (const double *)w,
                     (int)M, dots);
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(64), 0, s, ctl, (const double *)dots, g, yprev, rs);
  hipLaunchKernelGGL(k_scale, dim3(gM), dim3(kWG), 0, s, skip, (const double *)w, (const double *)&ctl->hn_inv,
                     (int)M, basis);
  chk();
  GCtl h{};
  for (int k0 = 0; k0 < m && !err; k0 += kGmresBatch) {
    const int k1 = std::min(m, k0 + kGmresBatch);
    for (int k = k0; k < k1; ++k) {
      const double *vk = basis + (size_t)k * M;
      double *wk = wbas + (size_t)k * M, *uk = ubas + (size_t)k * M;
      // w_k = M^{-1} D_reg z_k, u_k = V_dual w_k, Arnoldi vector M^{-1} u_k
      dreg(vk, t1);
      minv(t1, wk);
      vdual(wk, uk);
      minv(uk, w);
      if (inexact)
        hipLaunchKernelGGL(k_multidot, dim3(k + 1), dim3(kWG), 0, s, skip, (const double *)ubas, (int64_t)M,
                           (const double *)wk, (int)M, dots_gram);
      // two passes of classical Gram-Schmidt against v_0 .. v_k
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_multidot, dim3(k + 1), dim3(kWG), 0, s, skip, (const double *)basis, (int64_t)M,
                           (const double *)w, (int)M, dots);
        hipLaunchKernelGGL(k_gs_update, dim3(gM), dim3(kWG), 0, s, skip, (const double *)basis, (int64_t)M,
                           (const double *)dots, k + 1, (int)M, w);
        hipLaunchKernelGGL(k_gs_acc, dim3(blocks(k + 1)), dim3(kWG), 0, s, skip, (const double *)dots, k + 1, pass,
                           hacc);
      }
      hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, skip, (const double *)w, (int64_t)0,
                         (const double *)w, (int)M, dots);
      hipLaunchKernelGGL(k_gmres_rot, dim3(1), dim3(64), 0, s, ctl, (const double *)hacc, (const double *)dots, H, cs,
                         sn, g, k, rs, o.rtol, (int)inexact, (const double *)dots_gram, G, dots_y, yprev);
      if (inexact) {
        // x_k and eta(x_k) from its ZZ indicators
        hipLaunchKernelGGL(k_combine, dim3(gM), dim3(kWG), 0, s, skip, (const double *)wbas, (int64_t)M,
                           (const double *)dots_y, (const int32_t *)nullptr, k + 1, (int)M, x);
        hipLaunchKernelGGL(k_dual_zz, dim3(gN), dim3(kWG), 0, s, skip, (const double *)x, tris, area, diam, (int)N,
                           o.h_mode, eta2);
        hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, skip, (const double *)eta2, (int64_t)0, ones,
                           (int)N, dots_eta);
        hipLaunchKernelGGL(k_gmres_inexact, dim3(1), dim3(64), 0, s, ctl, (const double *)dots_eta,
                           o.inexact_lambda, k);
      }
      if (k + 1 < m)
        hipLaunchKernelGGL(k_scale, dim3(gM), dim3(kWG), 0, s, skip, (const double *)w, (const double *)&ctl->hn_inv,
                           (int)M, basis + (size_t)(k + 1) * M);
      chk();
    }
    // the device's decision after this batch
    if (hipMemcpyAsync(&h, ctl, sizeof(GCtl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      err = true;
    if (h.done) break;
  }
  if (err) return BC_EDEVICE;
  if (h.bad) return BC_EINVAL;
  // x = sum_i y_i w_i with y = R^{-1} g over the steps taken; Cap = (1/4pi) f^T x
  hipLaunchKernelGGL(k_gmres_final, dim3(1), dim3(64), 0, s, ctl, (const double *)H, (const double *)g, rs, m, yv,
                     nsteps);
  const int32_t *never = nsteps + 1;  // a flag that stays zero: the final kernels always run
  hipLaunchKernelGGL(k_combine, dim3(gM), dim3(kWG), 0, s, never, (const double *)wbas, (int64_t)M,
                     (const double *)yv, (const int32_t *)nsteps, 0, (int)M, x);
  hipLaunchKernelGGL(k_multidot, dim3(1), dim3(kWG), 0, s, never, f, (int64_t)0, (const double *)x, (int)M, dots);
  double capsum = 0.0;
  int32_t steps = 0;
  if (hipMemcpyAsync(&h, ctl, sizeof(GCtl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&capsum, dots, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&steps, nsteps, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return BC_EDEVICE;
  chk();
  if (err) return BC_EDEVICE;
  res->cap = capsum * kInv4Pi;
  res->rel_residual = h.rel;
  res->energy_step = inexact ? h.energy : 0.0;
  res->eta = inexact ? h.eta : 0.0;
  res->iters = steps;
  res->status = h.done ? BC_OK : BC_ENOCONV;
  res->stop = h.done ? h.stop : 0;
  res->reserved = 0;
  return BC_OK;
}

int launch_dual_zz(const void *ws, const int32_t *tris, int64_t N, int64_t M, int32_t restart, const double *x,
                   int h_mode, double *eta2, hipStream_t s) {
  const DualLayout L(N, M, restart);
  const char *b = static_cast<const char *>(ws);
  hipLaunchKernelGGL(k_dual_zz, dim3(blocks(N)), dim3(kWG), 0, s, (const int32_t *)nullptr, x, tris,
                     reinterpret_cast<const double *>(b + L.area),
                     reinterpret_cast<const double *>(b + L.diam), (int)N, h_mode, eta2);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
