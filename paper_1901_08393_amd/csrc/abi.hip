// Public C ABI of libbemcap: argument checks, workspace sizes, host-side
// mesh validation and the launch sequences.  Every numerical step runs in
// the HIP kernels of geometry.hip, assemble.hip, solve.hip and zz.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bc_internal.h"

namespace bc {

// Radon's 7-point rule of degree 5 on the reference triangle {s, t >= 0,
// s + t <= 1} (Stroud's T2:5-1): the centroid, and two orbits of three points
// with barycentric coordinates (1 - 2 b, b, b), b = (6 -+ sqrt 15) / 21, of
// weights (155 -+ sqrt 15) / 1200 and 9/40 at the centroid, all times the
// reference area 1/2.  A point is P0 + s (P1 - P0) + t (P2 - P0).
void radon7(double *s, double *t, double *w) {
  const double r = std::sqrt(15.0);
  s[0] = t[0] = 1.0 / 3.0;
  w[0] = 0.5 * 9.0 / 40.0;
  for (int o = 0; o < 2; ++o) {
    const double b = o == 0 ? (6.0 - r) / 21.0 : (6.0 + r) / 21.0, a = 1.0 - 2.0 * b;
    const double wo = 0.5 * (o == 0 ? (155.0 - r) : (155.0 + r)) / 1200.0;
    const double l1[3] = {b, a, b}, l2[3] = {b, b, a};
    for (int k = 0; k < 3; ++k) {
      s[1 + 3 * o + k] = l1[k];
      t[1 + 3 * o + k] = l2[k];
      w[1 + 3 * o + k] = wo;
    }
  }
}

// Gauss-Legendre nodes (ascending) and weights on [0, 1]: Newton's method
// on the Legendre polynomial P_n, evaluated by its three-term recurrence,
// started from cos(pi (k - 1/4) / (n + 1/2)).
void gauss_legendre01(int n, double *x, double *w) {
  std::vector<double> xs(n), ws(n);
  for (int k = 1; k <= n; ++k) {
    double z = std::cos(M_PI * (k - 0.25) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 1; j < n; ++j) {
        double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 1; j < n; ++j) {
      double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
      p0 = p1;
      p1 = p2;
    }
    double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
    dp = n * (z * pn - pm) / (z * z - 1.0);
    xs[k - 1] = z;
    ws[k - 1] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  std::vector<int> ord(n);
  for (int k = 0; k < n; ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return xs[a] < xs[b]; });
  for (int k = 0; k < n; ++k) {
    x[k] = 0.5 * (xs[ord[k]] + 1.0);
    w[k] = 0.5 * ws[ord[k]];
  }
}

SSTable ss_table(const bc_assembly_opts &o) {
  SSTable t{};
  for (int n = 1; n <= kSSMax; ++n) gauss_legendre01(n, t.x[n], t.w[n]);
  t.base = o.ss_order;
  t.edge = o.ss_order_edge;
  t.vertex = o.ss_order_vertex;
  t.sliver = o.ss_order_sliver;
  t.sliver_ratio = o.sliver_ratio;
  return t;
}

static bool opts_ok(const bc_assembly_opts *o) {
  if (!o) return false;
  if (o->far_order < 1 || o->far_order > 4) return false;
  if (o->ss_order < 1 || o->ss_order > kSSMax) return false;
  for (int32_t n : {o->ss_order_edge, o->ss_order_vertex, o->ss_order_sliver})
    if (n < 0 || n > kSSMax) return false;
  if (o->reserved != 0) return false;
  if (!(o->sliver_ratio >= 0.0) || !std::isfinite(o->sliver_ratio)) return false;
  if (o->ss_order_sliver > 0 && !(o->sliver_ratio > 0.0)) return false;
  if (o->precision != BC_FP64 && o->precision != BC_MIXED) return false;
  if (o->far_low != 0 && o->far_low != 1) return false;
  if (!(o->near_factor >= 0.0) || !std::isfinite(o->near_factor)) return false;
  if (o->precision == BC_FP64 && o->near_factor != 0.0) return false;
  return true;
}

static bool n_ok(int64_t N) { return N >= 1 && N <= (int64_t)1 << 20; }

}  // namespace bc

using namespace bc;

extern "C" {

int32_t bc_version(void) { return 10000; }

const char *bc_status_string(int32_t s) {
  switch (s) {
    case BC_OK: return "ok";
    case BC_EINVAL: return "invalid argument";
    case BC_EMESH: return "invalid mesh";
    case BC_ENOMEM: return "workspace too small";
    case BC_EDEVICE: return "HIP runtime error";
    case BC_ENOCONV: return "iteration limit reached before the tolerance";
    case BC_EBREAKDOWN: return "breakdown: matrix not positive definite";
    case BC_ETIMEOUT: return "cross-workgroup barrier timed out";
    case BC_RUNNING: return "running";
    default: return "unknown status";
  }
}

int64_t bc_matrix_ld(int64_t N) { return N < 0 ? 0 : ld_of(N); }

size_t bc_matrix_bytes(int64_t N, int32_t precision) {
  if (N < 0 || (precision != BC_FP64 && precision != BC_MIXED)) return 0;
  return (size_t)N * (size_t)ld_of(N) * (precision == BC_FP64 ? 8 : 4);
}

int32_t bc_mesh_check(const double *h_verts, int64_t M, const int32_t *h_tris, int64_t N, int64_t *h_bad_index) {
  auto fail = [&](int64_t k) {
    if (h_bad_index) *h_bad_index = k;
    return (int32_t)BC_EMESH;
  };
  if (h_bad_index) *h_bad_index = -1;
  if (!h_verts || !h_tris) return BC_EINVAL;
  if (N < 4 || M < 4 || N > ((int64_t)1 << 20) || M > ((int64_t)1 << 22)) return fail(-1);
  for (int64_t v = 0; v < M; ++v)
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(h_verts[3 * v + c])) return fail(v);
  std::vector<char> used(M, 0);
  for (int64_t e = 0; e < N; ++e) {
    int32_t a = h_tris[3 * e], b = h_tris[3 * e + 1], c = h_tris[3 * e + 2];
    if (a < 0 || b < 0 || c < 0 || a >= M || b >= M || c >= M) return fail(e);
    if (a == b || b == c || a == c) return fail(e);
    const double *p = h_verts + 3 * a, *q = h_verts + 3 * b, *r = h_verts + 3 * c;
    double ux = q[0] - p[0], uy = q[1] - p[1], uz = q[2] - p[2];
    double vx = r[0] - p[0], vy = r[1] - p[1], vz = r[2] - p[2];
    double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
    if (!(nx * nx + ny * ny + nz * nz > 0.0)) return fail(e);
    used[a] = used[b] = used[c] = 1;
  }
  for (int64_t v = 0; v < M; ++v)
    if (!used[v]) return fail(v);
  // welded: no two vertices with identical coordinates
  std::vector<int64_t> ord(M);
  for (int64_t v = 0; v < M; ++v) ord[v] = v;
  auto lt = [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(h_verts + 3 * a, h_verts + 3 * a + 3, h_verts + 3 * b, h_verts + 3 * b + 3);
  };
  std::sort(ord.begin(), ord.end(), lt);
  for (int64_t k = 1; k < M; ++k)
    if (std::equal(h_verts + 3 * ord[k - 1], h_verts + 3 * ord[k - 1] + 3, h_verts + 3 * ord[k])) return fail(ord[k]);
  // closed: every undirected edge in exactly two triangles
  std::vector<std::pair<int64_t, int64_t>> edges;
  edges.reserve(3 * N);
  for (int64_t e = 0; e < N; ++e)
    for (int k = 0; k < 3; ++k) {
      int64_t a = h_tris[3 * e + k], b = h_tris[3 * e + (k + 1) % 3];
      edges.emplace_back(std::min(a, b) * M + std::max(a, b), e);
    }
  std::sort(edges.begin(), edges.end());
  for (size_t k = 0; k < edges.size();) {
    size_t m = k;
    while (m < edges.size() && edges[m].first == edges[k].first) ++m;
    if (m - k != 2) return fail(edges[k].second);
    k = m;
  }
  return BC_OK;
}

size_t bc_mesh_workspace_bytes(int64_t N) { return N < 1 ? 0 : MeshLayout(N).total; }

size_t bc_pattern_bytes(int64_t N, int64_t nnz, int32_t precision) {
  if (N < 1 || nnz < 0 || (precision != BC_FP64 && precision != BC_MIXED)) return 0;
  return PatternLayout(N, nnz, precision).total;
}

int32_t bc_prepare(const double *d_verts, int64_t M, const int32_t *d_tris, int64_t N, const bc_assembly_opts *opts,
                   void *d_mesh_ws, size_t mesh_ws_bytes, bc_pattern_info *h_info, bc_stream stream) {
  if (!d_verts || !d_tris || !d_mesh_ws || !h_info || !n_ok(N) || M < 3 || !opts_ok(opts)) return BC_EINVAL;
  MeshLayout L(N);
  if (mesh_ws_bytes < L.total) return BC_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = launch_geometry(d_verts, d_tris, N, opts->far_order, d_mesh_ws, s);
  if (st != BC_OK) return st;
  st = launch_pattern(d_verts, d_tris, N, opts->near_factor, d_mesh_ws, nullptr, 0, opts->precision, false, s);
  if (st != BC_OK) return st;
  if (opts->precision == BC_MIXED) {
    st = launch_rsq_bias(d_mesh_ws, N, s);
    if (st != BC_OK) return st;
  }
  int64_t info[8] = {0};
  if (hipMemcpyAsync(info, static_cast<char *>(d_mesh_ws) + L.info, sizeof(info), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return BC_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return BC_EDEVICE;
  if (info[5] != 0) return BC_EINVAL;  // pattern larger than int32 indexing
  h_info->nnz = info[0];
  h_info->n_coincident = info[1];
  h_info->n_edge = info[2];
  h_info->n_vertex = info[3];
  h_info->n_near = info[4];
  return BC_OK;
}

int32_t bc_assemble(const double *d_verts, int64_t M, const int32_t *d_tris, int64_t N, const bc_assembly_opts *opts,
                    const void *d_mesh_ws, size_t mesh_ws_bytes, void *d_pattern, size_t pattern_bytes, int64_t nnz,
                    void *d_V, bc_stream stream) {
  if (!d_verts || !d_tris || !d_mesh_ws || !d_V || !n_ok(N) || M < 3 || !opts_ok(opts) || nnz < 0) return BC_EINVAL;
  if (nnz < N) return BC_EINVAL;  // every row holds at least its coincident entry
  if (!d_pattern) return BC_EINVAL;
  if (mesh_ws_bytes < MeshLayout(N).total) return BC_ENOMEM;
  if (pattern_bytes < PatternLayout(N, nnz, opts->precision).total) return BC_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = launch_pattern(d_verts, d_tris, N, opts->near_factor, d_mesh_ws, d_pattern, nnz, opts->precision, true, s);
  if (st != BC_OK) return st;
  return launch_assemble(d_mesh_ws, d_tris, d_verts, N, *opts, d_pattern, nnz, d_V, s);
}

int32_t bc_areas(const void *d_mesh_ws, int64_t N, double *d_area, bc_stream stream) {
  if (!d_mesh_ws || !d_area || !n_ok(N)) return BC_EINVAL;
  MeshLayout L(N);
  return hipMemcpyAsync(d_area, static_cast<const char *>(d_mesh_ws) + L.area, sizeof(double) * N,
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)) == hipSuccess
             ? BC_OK
             : BC_EDEVICE;
}

size_t bc_solve_workspace_bytes(int64_t N, int32_t precision) {
  if (N < 1 || (precision != BC_FP64 && precision != BC_MIXED)) return 0;
  return SolveLayout(N, precision).total;
}

int32_t bc_solve_workgroups(int64_t N) { return N < 1 ? 0 : solve_workgroups(N); }

int32_t bc_solve_capacity(int32_t precision) {
  if (precision != BC_FP64 && precision != BC_MIXED) return 0;
  int c = solve_capacity(precision);
  return c < 0 ? 0 : c;
}

size_t bc_batch_scratch_bytes(int32_t n_sys) { return n_sys < 1 ? 0 : align256(sizeof(SysDesc) * (size_t)n_sys); }

static bool solve_opts_ok(const bc_solve_opts *o) {
  return o && o->rtol >= 0.0 && std::isfinite(o->rtol) && o->inner_rtol > 0.0 && o->inner_rtol < 1.0 &&
         o->max_iter >= 1 && o->max_outer >= 1 && (o->jacobi == 0 || o->jacobi == 1) &&
         (o->x0_given == 0 || o->x0_given == 1) && o->cap_rtol >= 0.0 && o->cap_rtol < 1.0 && o->spin_limit >= 0 &&
         o->reserved == 0;
}

static SolveParams params_of(const bc_solve_opts *o, int32_t budget, int n_sys) {
  SolveParams p{};
  p.rtol = o->rtol;
  p.inner_rtol = o->inner_rtol;
  p.cap_rtol = o->cap_rtol;
  p.max_iter = o->max_iter;
  p.max_outer = o->max_outer;
  p.jacobi = o->jacobi;
  p.x0_given = o->x0_given;
  p.iter_budget = budget;
  p.spin_limit = o->spin_limit > 0 ? (uint32_t)o->spin_limit : 1u << 22;
  p.n_sys = n_sys;
  return p;
}

static int fill_desc(const bc_system &s, int wg_begin, SysDesc &d) {
  if (!s.V || !s.area || !s.sigma || !s.ws || !s.result || !n_ok(s.N) || s.nnz < 0) return BC_EINVAL;
  if (s.precision != BC_FP64 && s.precision != BC_MIXED) return BC_EINVAL;
  if (s.precision == BC_MIXED && s.nnz > 0 && !s.pattern) return BC_EINVAL;
  if (s.reserved != 0 || s.iter_budget < 0) return BC_EINVAL;
  if (s.N > (int64_t)kMaxBand * solve_workgroups(s.N)) return BC_EINVAL;  // rows per workgroup
  std::memset(&d, 0, sizeof(d));
  d.V = s.V;
  if (s.pattern && s.nnz > 0) {
    PatternLayout P(s.N, s.nnz, s.precision);
    const char *pb = static_cast<const char *>(s.pattern);
    d.prowptr = reinterpret_cast<const int32_t *>(pb + P.rowptr);
    d.pcol = reinterpret_cast<const int32_t *>(pb + P.col);
    d.pcorr = s.precision == BC_MIXED ? reinterpret_cast<const double *>(pb + P.corr) : nullptr;
  }
  d.area = s.area;
  d.sigma = s.sigma;
  d.ws = static_cast<char *>(s.ws);
  d.result = s.result;
  d.N = s.N;
  d.ld = ld_of(s.N);
  d.nnz = s.nnz;
  d.wg_begin = wg_begin;
  d.wg_count = solve_workgroups(s.N);
  d.start = s.start;
  d.budget = s.iter_budget;
  return BC_OK;
}

}  // extern "C"

namespace bc {
// bc_solve on a given workspace (also the body of the entry point whose
// workspace is the library's own device array).
int solve_one(const void *d_V, int64_t N, int32_t precision, const void *d_pattern, int64_t nnz, const double *d_area,
              double *d_sigma, const bc_solve_opts *opts, void *d_ws, size_t ws_bytes, bc_result *d_result,
              hipStream_t s) {
  if (!solve_opts_ok(opts)) return BC_EINVAL;
  if (precision != BC_FP64 && precision != BC_MIXED) return BC_EINVAL;
  if (!n_ok(N) || !d_ws) return BC_EINVAL;
  SolveLayout L(N, precision);
  // the descriptor lives after the control block, inside the workspace
  const size_t desc_off = sizeof(SolveCtl);
  static_assert(((sizeof(SolveCtl) + 63) & ~size_t(63)) + sizeof(SysDesc) <= 1024, "control block of 1 KB");
  if (ws_bytes < L.total) return BC_ENOMEM;
  bc_system sys{d_V, d_pattern, d_area, d_sigma, d_ws, d_result, N, nnz, precision, 1, 0, 0};
  SysDesc d;
  int st = fill_desc(sys, 0, d);
  if (st != BC_OK) return st;
  if (d.wg_count > solve_capacity(precision)) return BC_EDEVICE;
  SysDesc *dd = reinterpret_cast<SysDesc *>(static_cast<char *>(d_ws) + ((desc_off + 63) & ~size_t(63)));
  st = launch_set_desc(&d, 1, dd, s);
  if (st != BC_OK) return st;
  return launch_solve(precision, dd, 1, d.wg_count, params_of(opts, 0, 1), s);
}
}  // namespace bc

extern "C" {

int32_t bc_solve(const void *d_V, int64_t N, int32_t precision, const void *d_pattern, int64_t nnz,
                 const double *d_area, double *d_sigma, const bc_solve_opts *opts, void *d_ws, size_t ws_bytes,
                 bc_result *d_result, bc_stream stream) {
  return solve_one(d_V, N, precision, d_pattern, nnz, d_area, d_sigma, opts, d_ws, ws_bytes, d_result,
                   static_cast<hipStream_t>(stream));
}

int32_t bc_solve_batched(int32_t n_sys, const bc_system *h_sys, const bc_solve_opts *opts, int32_t iter_budget,
                         void *d_scratch, size_t scratch_bytes, bc_stream stream) {
  if (n_sys < 1 || !h_sys || !d_scratch || !solve_opts_ok(opts)) return BC_EINVAL;
  if (scratch_bytes < bc_batch_scratch_bytes(n_sys)) return BC_ENOMEM;
  const int32_t prec = h_sys[0].precision;
  std::vector<SysDesc> d(n_sys);
  int wg = 0;
  for (int k = 0; k < n_sys; ++k) {
    if (h_sys[k].precision != prec) return BC_EINVAL;
    int st = fill_desc(h_sys[k], wg, d[k]);
    if (st != BC_OK) return st;
    wg += d[k].wg_count;
  }
  if (wg > solve_capacity(prec)) return BC_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SysDesc *dd = static_cast<SysDesc *>(d_scratch);
  int st = launch_set_desc(d.data(), n_sys, dd, s);
  if (st != BC_OK) return st;
  return launch_solve(prec, dd, n_sys, wg, params_of(opts, iter_budget, n_sys), s);
}

int32_t bc_capacity(const double *d_sigma, const double *d_area, int64_t N, double *d_cap, bc_stream stream) {
  if (!d_sigma || !d_area || !d_cap || !n_ok(N)) return BC_EINVAL;
  return launch_capacity(d_sigma, d_area, N, d_cap, static_cast<hipStream_t>(stream));
}

size_t bc_residual_workspace_bytes(int64_t N, int64_t nnz) {
  if (!n_ok(N) || nnz < N) return 0;
  return residual_workspace_bytes(N, nnz);
}

int32_t bc_residual_indicators(const double *d_verts, const int32_t *d_tris, int64_t N, const bc_assembly_opts *opts,
                               const void *d_mesh_ws, const void *d_pattern, int64_t nnz, const double *d_sigma,
                               double *d_mu2, double *d_moments, void *d_ws, size_t ws_bytes, bc_stream stream) {
  if (!d_verts || !d_tris || !d_mesh_ws || !d_pattern || !d_sigma || !d_mu2 || !d_ws) return BC_EINVAL;
  if (!n_ok(N) || nnz < N || !opts_ok(opts)) return BC_EINVAL;
  if (ws_bytes < residual_workspace_bytes(N, nnz)) return BC_ENOMEM;
  return launch_residual(d_verts, N, *opts, d_mesh_ws, d_pattern, nnz, d_sigma, d_mu2, d_moments, d_ws,
                         static_cast<hipStream_t>(stream));
}

int32_t bc_zz_indicators(const int32_t *d_tris, int64_t N, const void *d_mesh_ws, const void *d_pattern, int64_t nnz,
                         const double *d_sigma, int32_t h_mode, double *d_eta2, bc_stream stream) {
  if (!d_tris || !d_mesh_ws || !d_pattern || !d_sigma || !d_eta2 || !n_ok(N) || nnz < N) return BC_EINVAL;
  if (h_mode != 0 && h_mode != 1) return BC_EINVAL;
  return launch_zz(d_tris, N, d_mesh_ws, d_pattern, nnz, d_sigma, h_mode, d_eta2, static_cast<hipStream_t>(stream));
}

static bool matvec_ok(int64_t N, int32_t precision, int32_t nrhs) {
  return n_ok(N) && (((precision == BC_FP64 || precision == BC_F32_F64) && (nrhs == 1 || nrhs == 3)) ||
                     (precision == BC_MIXED && nrhs == 1));
}

size_t bc_matvec_workspace_bytes(int64_t N, int32_t precision, int32_t nrhs) {
  if (!matvec_ok(N, precision, nrhs)) return 0;
  return MatvecLayout(N, precision, nrhs).total;
}

int32_t bc_matvec(const void *d_V, int64_t N, int32_t precision, int32_t nrhs, const void *d_x, void *d_y,
                  void *d_ws, size_t ws_bytes, bc_stream stream) {
  if (!d_V || !d_x || !d_y || !d_ws || !matvec_ok(N, precision, nrhs)) return BC_EINVAL;
  if (N > (int64_t)kMaxBand * solve_workgroups(N)) return BC_EINVAL;
  if (ws_bytes < MatvecLayout(N, precision, nrhs).total) return BC_ENOMEM;
  return launch_matvec(precision, d_V, N, nrhs, d_x, d_y, d_ws, static_cast<hipStream_t>(stream));
}

static bool dual_sizes_ok(int64_t N, int64_t M, int32_t restart) {
  return n_ok(N) && M >= 4 && M <= 3 * N && restart >= 1 && restart <= 1000 && 6 * N <= (int64_t)1 << 20 &&
         6 * N <= (int64_t)kMaxBand * solve_workgroups(6 * N);
}

size_t bc_dual_workspace_bytes(int64_t N, int64_t M, int32_t restart) {
  if (!dual_sizes_ok(N, M, restart)) return 0;
  return DualLayout(N, M, restart).total;
}

int32_t bc_dual_setup(const double *d_verts, int64_t M, const int32_t *d_tris, int64_t N, const int32_t *d_iptr,
                      const int32_t *d_itri, void *d_ws, size_t ws_bytes, int32_t restart, bc_stream stream) {
  if (!d_verts || !d_tris || !d_iptr || !d_itri || !d_ws || !dual_sizes_ok(N, M, restart)) return BC_EINVAL;
  if (ws_bytes < DualLayout(N, M, restart).total) return BC_ENOMEM;
  return launch_dual_setup(d_verts, d_tris, N, M, d_iptr, d_itri, d_ws, restart, static_cast<hipStream_t>(stream));
}

int32_t bc_dual_solve(const void *d_Vbary, int32_t precision, const void *d_pattern, int64_t nnz,
                      const int32_t *d_tris, int64_t N, int64_t M, const int32_t *d_iptr, const int32_t *d_itri,
                      const int32_t *d_icor, void *d_ws, size_t ws_bytes, const bc_dual_opts *opts, double *d_x,
                      bc_dual_result *h_result, bc_stream stream) {
  if (!d_Vbary || !d_tris || !d_iptr || !d_itri || !d_icor || !d_ws || !opts || !d_x || !h_result) return BC_EINVAL;
  if (precision != BC_FP64 && precision != BC_MIXED) return BC_EINVAL;
  if (precision == BC_MIXED && (!d_pattern || nnz < 0)) return BC_EINVAL;
  if (!dual_sizes_ok(N, M, opts->restart)) return BC_EINVAL;
  if (!(opts->rtol > 0.0) || !std::isfinite(opts->rtol) || opts->max_iter < 1 || opts->max_iter > opts->restart ||
      opts->jacobi_sweeps < 0 || opts->jacobi_sweeps > 1000 || (opts->h_mode != 0 && opts->h_mode != 1) ||
      !(opts->inexact_lambda >= 0.0) || !std::isfinite(opts->inexact_lambda))
    return BC_EINVAL;
  if (ws_bytes < DualLayout(N, M, opts->restart).total) return BC_ENOMEM;
  return run_dual_solve(d_Vbary, precision, d_pattern, nnz, d_tris, N, M, d_iptr, d_itri, d_icor, d_ws, *opts, d_x,
                        h_result, static_cast<hipStream_t>(stream));
}

int32_t bc_dual_zz(const void *d_ws, size_t ws_bytes, const int32_t *d_tris, int64_t N, int64_t M, int32_t restart,
                   const double *d_x, int32_t h_mode, double *d_eta2, bc_stream stream) {
  if (!d_ws || !d_tris || !d_x || !d_eta2 || !dual_sizes_ok(N, M, restart) || (h_mode != 0 && h_mode != 1))
    return BC_EINVAL;
  if (ws_bytes < DualLayout(N, M, restart).total) return BC_ENOMEM;
  return launch_dual_zz(d_ws, d_tris, N, M, restart, d_x, h_mode, d_eta2, static_cast<hipStream_t>(stream));
}

}  // extern "C"
