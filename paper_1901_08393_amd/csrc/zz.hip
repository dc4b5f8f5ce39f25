// ZZ-type error indicators for the P0 solution (eq. "zz:T", Section 2.4):
//
//   eta(T)^2 = h_T || sigma_T - I sigma ||^2_{L2(T)}.
//
// The nodal value of I sigma at a vertex z is the area-weighted mean of
// sigma over the elements containing z.  Those elements are exactly the
// entries of row i of the pattern (classes vertex / edge / coincident) that
// contain z, for any element i containing z; rows are sorted by column, so
// every element sharing z sums the same terms in the same (increasing
// element) order and obtains the bit-identical nodal value, without atomics
// or a vertex-to-element table.  On T the difference sigma_T - I sigma is
// linear with vertex values -d_k, so
//   || . ||^2 = |T| / 12 ((d1 + d2 + d3)^2 + d1^2 + d2^2 + d3^2).
#include "bc_internal.h"

namespace bc {

// One wavefront per element i: its lanes load the entries of row i once
// (class, column, the column element's vertices, area and sigma), and for each
// vertex z of T_i a ballot selects the elements containing z; lane order is
// column order, so adding the selected lanes in increasing order gives the
// sums of the plain row loop, term by term.
constexpr int kZZRows = kWG / 64;  // elements per workgroup

__global__ __launch_bounds__(kWG) void k_zz(const int4 *__restrict__ tri4, const double4 *__restrict__ cen4,
                                            const double *__restrict__ area, const int32_t *__restrict__ prowptr,
                                            const int32_t *__restrict__ pcol, const int32_t *__restrict__ pkind,
                                            const double *__restrict__ sigma, int N, int h_mode,
                                            double *__restrict__ eta2) {
  // no contraction: the sums round like the plain expressions
#pragma clang fp contract(off)
  const int lane = (int)threadIdx.x & 63;
  const int i = (int)blockIdx.x * kZZRows + ((int)threadIdx.x >> 6);
  if (i >= N) return;  // wavefront-uniform
  const int4 ti = tri4[i];
  const int zs[3] = {ti.x, ti.y, ti.z};
  double num[3] = {0.0, 0.0, 0.0}, den[3] = {0.0, 0.0, 0.0};
  const int e0 = prowptr[i], e1 = prowptr[i + 1];
  for (int c = e0; c < e1; c += 64) {
    const int e = c + lane;
    bool has[3] = {false, false, false};
    double aj = 0.0, asj = 0.0;
    if (e < e1 && pkind[e] != kNear) {
      const int j = pcol[e];
      const int4 tj = tri4[j];
      aj = area[j];
      asj = aj * sigma[j];
      for (int k = 0; k < 3; ++k) has[k] = tj.x == zs[k] || tj.y == zs[k] || tj.z == zs[k];
    }
    for (int k = 0; k < 3; ++k) {
      uint64_t m = __ballot(has[k]);
      while (m) {  // increasing lanes: increasing columns
        const int l = __builtin_ctzll(m);
        m &= m - 1;
        num[k] += lane_f(asj, l);
        den[k] += lane_f(aj, l);
      }
    }
  }
  if (lane != 0) return;
  const double si = sigma[i];
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = num[k] / den[k] - si;
  const double s = d[0] + d[1] + d[2];
  const double l2 = area[i] / 12.0 * (s * s + d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double h = h_mode == 0 ? sqrt(cen4[i].w) : sqrt(area[i]);
  eta2[i] = h * l2;
}

int launch_zz(const int32_t *tris, int64_t N, const void *mesh_ws, const void *pattern, int64_t nnz,
              const double *sigma, int h_mode, double *eta2, hipStream_t s) {
  (void)tris;
  const MeshView m = mesh_view(mesh_ws, N);
  PatternLayout P(N, nnz, BC_FP64);  // offsets of rowptr/col/kind do not depend on precision
  const char *pb = static_cast<const char *>(pattern);
  hipLaunchKernelGGL(k_zz, dim3((unsigned)((N + kZZRows - 1) / kZZRows)), dim3(kWG), 0, s, m.tri4, m.cen4, m.area,
                     reinterpret_cast<const int32_t *>(pb + P.rowptr), reinterpret_cast<const int32_t *>(pb + P.col),
                     reinterpret_cast<const int32_t *>(pb + P.kind), sigma, (int)N, h_mode, eta2);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
