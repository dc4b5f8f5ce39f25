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

__global__ __launch_bounds__(kWG) void k_zz(const int4 *__restrict__ tri4, const double4 *__restrict__ cen4,
                                            const double *__restrict__ area, const int32_t *__restrict__ prowptr,
                                            const int32_t *__restrict__ pcol, const int32_t *__restrict__ pkind,
                                            const double *__restrict__ sigma, int N, int h_mode,
                                            double *__restrict__ eta2) {
  // no contraction: the sums round like the plain expressions
#pragma clang fp contract(off)
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i >= N) return;
  const int4 ti = tri4[i];
  const int zs[3] = {ti.x, ti.y, ti.z};
  double d[3];
  const double si = sigma[i];
  for (int k = 0; k < 3; ++k) {
    const int z = zs[k];
    double num = 0.0, den = 0.0;
    for (int e = prowptr[i]; e < prowptr[i + 1]; ++e) {
      if (pkind[e] == kNear) continue;
      const int j = pcol[e];
      const int4 tj = tri4[j];
      if (tj.x == z || tj.y == z || tj.z == z) {
        num += area[j] * sigma[j];
        den += area[j];
      }
    }
    d[k] = num / den - si;
  }
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
  hipLaunchKernelGGL(k_zz, dim3((int)((N + kWG - 1) / kWG)), dim3(kWG), 0, s, m.tri4, m.cen4, m.area,
                     reinterpret_cast<const int32_t *>(pb + P.rowptr), reinterpret_cast<const int32_t *>(pb + P.col),
                     reinterpret_cast<const int32_t *>(pb + P.kind), sigma, (int)N, h_mode, eta2);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
