// Dense assembly of the P0 Galerkin matrix of the single-layer operator
// (Appendix A, eq. "discreteform:residual"; kernel 1/(4 pi |x - y|) of
// eq. "strongform"):
//
//   V[i][j] = (1/4pi) int_{T_i} int_{T_j} 1/|x - y| dy dx.
//
// k_far64 / k_far32: every pair i <= j with the collapsed Q-point Gauss rule
//   on both triangles (Q^2 point pairs).  One workgroup per 64 x 64 tile of
//   the upper block triangle; lanes own columns j and keep that element's Q
//   points in registers; the 16 rows of a wave are read with uniform
//   (scalar) loads.  The value is stored at (i, j) and mirrored to (j, i).
//   ALU-bound.  In mixed precision with Q = 16 the tiles are split by class
//   (lists built by bc_prepare): k_far32 takes the near and diagonal tiles,
//   k_far32m the separated ones, where the squared distances of 16 x 16
//   element pairs are one matrix-core product per point pair (the distant
//   tiles, at least 8 element diameters apart, with Radon's 7-point rule).
// k_sparse: one wavefront per pattern entry with j >= i: touching pairs with
//   the Sauter-Schwab-type rules, near pairs (mixed precision) with the
//   regular rule, both in FP64; overwrites the far-field value.  In mixed
//   precision it also stores the FP64 correction V64 - (double)(float)V64 at
//   both (i, j) and (j, i) of the pattern.
// k_pad: zeros in the padding columns N..ld-1.
#include <algorithm>
#include <type_traits>

#include "bc_internal.h"

namespace bc {

// ----------------------------------------------------------------- far field
// FP64 far field: V_ij = (1/4pi) sum_a sum_b W_a W_b / |x_a - y_b| over the
// tensor rule's points (absolute coordinates, FP64), the inverse square root
// refined by one Newton step (rsqrt64_far2).  Tiles at least kSepFar block
// diameters apart expand -r^2 = -|x|^2 - |y|^2 + 2 x.y about the column
// element's centroid; closer tiles form differences.
// Inverse square root for the FP64 far field: the hardware estimate y and one
// Newton step, y (3 - x y^2) / 2, returned without the factor 1/2, which the
// column weights carry: two multiplications and one FMA.  Measured over
// log-uniform inputs against 1/sqrt(x): at most 38 ulp (4.3e-15 relative),
// mean -1.5e-16, the same as the form y + (y/2)(1 - x y^2), which needs one
// FMA more.  A far entry sums 256 such terms with positive weights, so its
// relative error stays below 5e-15.  The kernel is bound by instruction
// issue: per point pair four FP64 operations for -r^2, the estimate (3.2
// FMA-equivalents, measured), three for the Newton step and one to accumulate.
// (The cubic step of rsqrt64, kept for the singular and near rules, costs two
// more FP64 operations per point pair.)
__device__ __forceinline__ double rsqrt64_far2(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * __builtin_fma(-(x * y), y, 3.0);
}

// One 64 x 64 tile (I, J), I <= J, with the Q-point rule whose points sit
// STRIDE apart per element in the row table qpA ([N][STRIDE]) and in the
// column table qpS ([(b*4+c)][N]).  FORM: 0 the form chosen per tile
// (expansion on separated tiles), 1 differences, 2 the expansion (tiles known
// to be separated).  A kernel with one form schedules better than one that
// branches between them per tile.
template <int Q, int STRIDE, int FORM>
__device__ __forceinline__ void far64_tile(int I, int J, const double4 *__restrict__ qpA,
                                           const double *__restrict__ qpS, const double4 *__restrict__ cen4,
                                           const double *__restrict__ bbox, int N, int64_t ld, double *__restrict__ V) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = J * 64 + lane;
  const bool jv = j < N;
  const int jj = jv ? j : N - 1;
  const bool sep = FORM == 0 ? far_separated(bbox, I, J) : FORM == 2;
  // column element's points relative to its centroid (separated tiles) or
  // absolute (close tiles)
  const double4 cj = cen4[jj];
  const double ox = sep ? cj.x : 0.0, oy = sep ? cj.y : 0.0, oz = sep ? cj.z : 0.0;
  double yx[Q], yy[Q], yz[Q], yw[Q], yn[Q];
#pragma unroll
  for (int b = 0; b < Q; ++b) {
    yx[b] = qpS[(size_t)(b * 4 + 0) * N + jj] - ox;
    yy[b] = qpS[(size_t)(b * 4 + 1) * N + jj] - oy;
    yz[b] = qpS[(size_t)(b * 4 + 2) * N + jj] - oz;
    yw[b] = 0.5 * qpS[(size_t)(b * 4 + 3) * N + jj];  // the Newton step's 1/2
    yn[b] = -(yx[b] * yx[b] + yy[b] * yy[b] + yz[b] * yz[b]);
  }
  const int i0 = I * 64 + w * 16;
  auto row = [&](auto SEP, int i) {
    const double4 *xa = qpA + (size_t)i * STRIDE;
    double acc = 0.0;
#pragma unroll 2
    for (int a = 0; a < Q; ++a) {
      const double4 p = xa[a];
      const double ex = p.x - ox, ey = p.y - oy, ez = p.z - oz;
      const double ne = -(ex * ex + ey * ey + ez * ez);
      const double tx = 2.0 * ex, ty = 2.0 * ey, tz = 2.0 * ez;
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        double c;  // -r^2
        if constexpr (decltype(SEP)::value) {
          c = __builtin_fma(tz, yz[b], __builtin_fma(ty, yy[b], __builtin_fma(tx, yx[b], ne + yn[b])));
        } else {
          const double dx = ex - yx[b], dy = ey - yy[b], dz = ez - yz[b];
          c = -(dx * dx + dy * dy + dz * dz);
        }
        s = __builtin_fma(yw[b], rsqrt64_far2(-c), s);
      }
      acc = __builtin_fma(p.w, s, acc);
    }
    if (jv && j >= i) {
      const double v = acc * kInv4Pi;
      V[(size_t)i * ld + j] = v;
      V[(size_t)j * ld + i] = v;
    }
  };
  for (int k = 0; k < 16; ++k) {
    const int i = i0 + k;
    if (i >= N) break;
    if constexpr (FORM == 1) {
      row(std::false_type{}, i);
    } else if constexpr (FORM == 2) {
      row(std::true_type{}, i);
    } else {
      if (sep) row(std::true_type{}, i); else row(std::false_type{}, i);
    }
  }
}

// One workgroup per tile of the upper block triangle, or (LIST) the tiles of
// one list from bc_prepare, visited grid-stride.
template <int Q, int STRIDE, bool LIST, int FORM>
__global__ __launch_bounds__(kWG) void k_far64(const double4 *__restrict__ qpA, const double *__restrict__ qpS,
                                               const double4 *__restrict__ cen4, const double *__restrict__ bbox,
                                               const int32_t *__restrict__ cnt, const int32_t *__restrict__ list,
                                               int N, int64_t ld, double *__restrict__ V) {
  int I, J;
  if (!LIST) {
    tile_of(blockIdx.x, I, J);
    far64_tile<Q, STRIDE, FORM>(I, J, qpA, qpS, cen4, bbox, N, ld, V);
    return;
  }
  const int nt = (int)far_tiles(N), n = min(*cnt, nt);
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int t = list[q];
    if (t < 0 || t >= nt) continue;  // lists from another mesh: nothing out of range
    tile_of(t, I, J);
    far64_tile<Q, STRIDE, FORM>(I, J, qpA, qpS, cen4, bbox, N, ld, V);
  }
}

// FP32 far field.  The point offsets are relative to the element centroid
// and the weights are those of the reference triangle; the entry is
//   (float)( (double)S_ij * 4 |T_i| |T_j| * scale / (1 + beta) ),
//   S_ij = sum_a w_a sum_b w_b rsq(r_ab^2)   (FP32),
// with scale = (1/4pi) (sum w / sum fl(w))^2 formed in FP64 on the host and
// beta the mean relative error of the hardware inverse square root, measured
// on the device (k_rsq_bias), so that neither 1/(4pi), the weights nor the
// inverse square root carry an FP32 error that is the same for every entry
// (such a common error would shift the capacity by the same relative
// amount).  What remains per point pair is rounding of either sign, about one
// FP32 ulp, which the 256-term sums and the FP32 storage of V dominate.
//
// The vector kernel (k_far32) forms r^2 from the differences e - y, e =
// c_i - c_j + x_a and y the offset of y_b from c_j: three subtractions and
// three multiply-adds per point pair.  Its tiles are the near and diagonal
// ones and the separated tiles whose column block is not compact; separated
// compact tiles go to the matrix cores (k_far32m).  (Expanding -r^2 =
// -|e|^2 - |y|^2 + 2 e.y on the separated tiles here would save two
// operations per point pair, but the kernel with both forms behind a branch
// per tile was slower on every tile: L5 sphere assembly 3.45 against 3.31 ms
// with differences alone.)

// Mean relative error of v_rsq_f32 over inputs spread log-uniformly over
// [1, 4) (the error depends only on the mantissa and the exponent's parity,
// as scaling x by 4 scales rsq(x) by exactly 1/2): 2^16 inputs
// x_k = 2^(2 (k + 1/2) / 2^16), errors y sqrt(x) - 1 formed in FP64.
// k_rsq_part: kRsqParts workgroups, each the fixed-order sum of its
// contiguous range of k into out[1 + part]; k_rsq_bias: the parts added in
// order into out[0] and divided by the count.  Written by bc_prepare (mixed
// precision) into the caller's mesh workspace, where the FP32 far-field
// kernels read it.  (One workgroup of 1024 threads took 29 us.)
constexpr int kRsqSamples = 1 << 16;
constexpr int kRsqWG = 256;
static_assert(kRsqSamples % (kRsqParts * kRsqWG) == 0, "whole rounds per part");

__global__ __launch_bounds__(kRsqWG) void k_rsq_part(double *__restrict__ out) {
  __shared__ double part[kRsqWG];
  constexpr int per = kRsqSamples / kRsqParts;
  const int k0 = (int)blockIdx.x * per;
  double s = 0.0;
  for (int k = k0 + (int)threadIdx.x; k < k0 + per; k += kRsqWG) {
    const float x = (float)exp2(2.0 * (k + 0.5) / kRsqSamples);
    const double y = (double)__builtin_amdgcn_rsqf(x);
    s += y * sqrt((double)x) - 1.0;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  // fixed-order tree over the workgroup's partial sums
  for (int h = kRsqWG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[1 + blockIdx.x] = part[0];
}

__global__ __launch_bounds__(64) void k_rsq_bias(double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int p = 0; p < kRsqParts; ++p) s += out[1 + p];
  out[0] = s / kRsqSamples;
}

int launch_rsq_bias(void *mesh_ws, int64_t N, hipStream_t s) {
  MeshLayout L(N);
  double *out = reinterpret_cast<double *>(static_cast<char *>(mesh_ws) + L.rsqb);
  hipLaunchKernelGGL(k_rsq_part, dim3(kRsqParts), dim3(kRsqWG), 0, s, out);
  hipLaunchKernelGGL(k_rsq_bias, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

template <int Q>
__device__ __forceinline__ void far32_tile(int I, int J, const float4 *__restrict__ qpA,
                                           const float *__restrict__ qpS, const double4 *__restrict__ cen4,
                                           const double *__restrict__ area, const double *__restrict__ rsqb,
                                           double scale, int N, int64_t ld, float *__restrict__ V) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = J * 64 + lane;
  const bool jv = j < N;
  const int jj = jv ? j : N - 1;
  float vx[Q], vy[Q], vz[Q], vw[Q];
#pragma unroll
  for (int b = 0; b < Q; ++b) {
    vx[b] = qpS[(size_t)(b * 4 + 0) * N + jj];
    vy[b] = qpS[(size_t)(b * 4 + 1) * N + jj];
    vz[b] = qpS[(size_t)(b * 4 + 2) * N + jj];
    vw[b] = qpS[(size_t)(b * 4 + 3) * N + jj];
  }
  const double4 cj = cen4[jj];
  const double aj = 4.0 * area[jj] * (scale / (1.0 + *rsqb));
  const int i0 = I * 64 + w * 16;
  auto row = [&](int i) {
    const double4 ci = cen4[i];
    // centroid difference formed in FP64 and kept as hi + lo floats, so that
    // each point offset e = D_hi + (x_a + D_lo) is one rounding of D + x_a.
    // Rounding D alone would give every pair with the same D the same error;
    // on lattice-like meshes (boxes) such errors share their sign and would
    // shift the capacity by up to 1e-8.
    const double dX = ci.x - cj.x, dY = ci.y - cj.y, dZ = ci.z - cj.z;
    const float Dx = (float)dX, Dy = (float)dY, Dz = (float)dZ;
    const float Lx = (float)(dX - (double)Dx), Ly = (float)(dY - (double)Dy), Lz = (float)(dZ - (double)Dz);
    const float4 *ua = qpA + (size_t)i * kQMax;
    float acc = 0.f;
#pragma unroll 2
    for (int a = 0; a < Q; ++a) {
      const float4 p = ua[a];
      const float ex = Dx + (p.x + Lx), ey = Dy + (p.y + Ly), ez = Dz + (p.z + Lz);
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        const float dx = ex - vx[b], dy = ey - vy[b], dz = ez - vz[b];
        s = __builtin_fmaf(vw[b], __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz), s);
      }
      acc = __builtin_fmaf(p.w, s, acc);
    }
    if (jv && j >= i) {
      const float v = (float)((double)acc * (area[i] * aj));
      V[(size_t)i * ld + j] = v;
      V[(size_t)j * ld + i] = v;
    }
  };
  for (int k = 0; k < 16; ++k) {
    const int i = i0 + k;
    if (i >= N) break;
    row(i);
  }
}

// One workgroup per tile of the upper block triangle, or (LIST) the tiles of
// one list, visited grid-stride.
template <int Q, bool LIST>
__global__ __launch_bounds__(kWG) void k_far32(const float4 *__restrict__ qpA, const float *__restrict__ qpS,
                                               const double4 *__restrict__ cen4, const double *__restrict__ area,
                                               const int32_t *__restrict__ cnt, const int32_t *__restrict__ list,
                                               const double *__restrict__ rsqb, double scale, int N, int64_t ld,
                                               float *__restrict__ V) {
  int I, J;
  if (!LIST) {
    tile_of(blockIdx.x, I, J);
    far32_tile<Q>(I, J, qpA, qpS, cen4, area, rsqb, scale, N, ld, V);
    return;
  }
  const int nt = (int)far_tiles(N), n = min(*cnt, nt);
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int t = list[q];
    if (t < 0 || t >= nt) continue;  // lists from another mesh: nothing out of range
    tile_of(t, I, J);
    far32_tile<Q>(I, J, qpA, qpS, cen4, area, rsqb, scale, N, ld, V);
  }
}

// FP32 reference weights of a far rule (the same for every element).
struct FarWeights {
  float w[kQMax];
};

// FP32 far field of separated tiles (I < J, at least kSepFar block diameters
// apart) on the matrix cores.  A wavefront takes 16 rows of a tile and its
// four 16-column sub-blocks in turn (the row operands, which depend on the
// column block only, are formed once for the four); for each sub-block and
// each pair of points (a, b) one v_mfma_f32_16x16x4f32 forms
//   -r^2 = 2 e.y - |e|^2 - |y|^2        for all 16 x 16 element pairs,
// A[i][k] = (2 e_x, 2 e_y, 2 e_z, -|e|^2) of point a of row element i,
// B[k][j] = (y_x, y_y, y_z, 1) of point b of column element j, C = -|y|^2,
// with e and y relative to the centre of the column block's bounding box
// (formed in FP64 and rounded once, like the norms).  Lane l then holds
// -r^2 for rows 4 (l / 16) .. + 3 and column l % 16, and only the inverse
// square roots and the weighted sums remain on the vector ALU.  The sums,
// weights, scale and bias correction are those of k_far32.  QP points per
// element: the 4 x 4 rule (16) or Radon's rule of distant tiles (kQLow); the
// row points from the FP64 table qpA (QP per element), the column operands
// from qpB (per point, relative to the column element's own block, which is
// the column block; tabulated by bc_prepare).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int QP>
__device__ __forceinline__ void far32m_tile(int I, int J, int rsb, const double4 *__restrict__ qpA,
                                            const float *__restrict__ qpB, const FarWeights &fw,
                                            const double *__restrict__ area, const double *__restrict__ bbox,
                                            const double *__restrict__ rsqb, double scale, int N, int64_t ld,
                                            float *__restrict__ V) {
  static_assert(QP == 16 || QP == kQLow, "far rule of 16 or kQLow points");
  const int lane = (int)__lane_id();
  const int i0 = I * 64 + 16 * rsb;
  if (i0 >= N) return;  // the wavefront's rows lie past the end (wavefront-uniform)
  const int k = lane >> 4;
  const int ia = min(i0 + (lane & 15), N - 1);
  const double *bj = bbox + 8 * J;
  const double fx = 0.5 * (bj[0] + bj[3]), fy = 0.5 * (bj[1] + bj[4]), fz = 0.5 * (bj[2] + bj[5]);
  // the row operands relative to the column block's box centre: the same for
  // the tile's four column sub-blocks, which this wavefront takes in turn
  float av[QP];
#pragma unroll
  for (int a = 0; a < QP; ++a) {
    const double4 p = qpA[(size_t)ia * QP + a];
    const double ex = p.x - fx, ey = p.y - fy, ez = p.z - fz;
    av[a] = (float)(k == 0 ? 2.0 * ex : (k == 1 ? 2.0 * ey : (k == 2 ? 2.0 * ez : -(ex * ex + ey * ey + ez * ez))));
  }
  const double sb = scale / (1.0 + *rsqb);
  const int ib = i0 + 4 * k;
#pragma unroll 1
  for (int csb = 0; csb < 4; ++csb) {
    const int j0 = J * 64 + 16 * csb;
    if (j0 >= N) break;  // wavefront-uniform
    const int jb = min(j0 + (lane & 15), N - 1);
    float S[4] = {0.f, 0.f, 0.f, 0.f};
    // the column point relative to the column block's box centre, and its
    // squared norm (tabulated by bc_prepare); the next point's pair is loaded
    // while this one is used, so that no iteration waits for its own loads
    auto col_b = [&](int b) { return k < 3 ? qpB[(size_t)(b * 4 + k) * N + jb] : 1.0f; };
    auto col_n = [&](int b) { return qpB[(size_t)(b * 4 + 3) * N + jb]; };
    float bv_next = col_b(0), yn_next = col_n(0);
    for (int b = 0; b < QP; ++b) {
      const float bv = bv_next, yn = yn_next;
      if (b + 1 < QP) {
        bv_next = col_b(b + 1);
        yn_next = col_n(b + 1);
      }
      const float wb = fw.w[b];
      const v4f C = {-yn, -yn, -yn, -yn};
      float Sb[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int a = 0; a < QP; ++a) {
        const v4f D = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv, C, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) Sb[r] = __builtin_fmaf(fw.w[a], __builtin_amdgcn_rsqf(-D[r]), Sb[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) S[r] = __builtin_fmaf(wb, Sb[r], S[r]);
    }
    const int j = j0 + (lane & 15);
    if (j < N) {
      const double aj = 4.0 * area[j] * sb;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = ib + r < N ? (float)((double)S[r] * (area[ib + r] * aj)) : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (ib + r < N) V[(size_t)(ib + r) * ld + j] = v[r];
      // the mirrored entries (j, ib .. ib + 3) are consecutive in row j
      if (ib + 3 < N) {
        *reinterpret_cast<float4 *>(V + (size_t)j * ld + ib) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        for (int r = 0; r < 4; ++r)
          if (ib + r < N) V[(size_t)j * ld + ib + r] = v[r];
      }
    }
  }
}

// The tiles of one list, grid-stride, one tile per four wavefronts (one per
// 16-row sub-block; no workgroup barrier: a wavefront that has nothing to do
// in a tile goes on to the next).  Workgroups of kFarMWG threads, kFarMGrid
// per CU in the grid (L5 sphere, mixed assembly: 3.49 ms with 512 x 4, 3.53
// with 1024 x 2, 3.77 with 256 x 8; 72 registers allow 7 wavefronts per SIMD).
constexpr int kFarMWG = 512;
constexpr int kFarMGrid = 4;
template <int QP>
__global__ __launch_bounds__(kFarMWG) void k_far32m(const double4 *__restrict__ qpA, const float *__restrict__ qpB,
                                                    FarWeights fw, const double *__restrict__ area,
                                                    const double *__restrict__ bbox, const int32_t *__restrict__ cnt,
                                                    const int32_t *__restrict__ list, const double *__restrict__ rsqb,
                                                    double scale, int N, int64_t ld, float *__restrict__ V) {
  constexpr int TPW = kFarMWG / 256;  // tiles per workgroup pass
  const int nt = (int)far_tiles(N), n = min(*cnt, nt);
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  for (int q = (int)blockIdx.x * TPW + (w >> 2); q < n; q += (int)gridDim.x * TPW) {
    const int t = list[q];
    if (t < 0 || t >= nt) continue;  // lists from another mesh: nothing out of range
    int I, J;
    tile_of(t, I, J);
    far32m_tile<QP>(I, J, w & 3, qpA, qpB, fw, area, bbox, rsqb, scale, N, ld, V);
  }
}

// ------------------------------------------------------- touching and near
// One pattern entry (i, j), j >= i: touching pairs with the singular rule of
// the pair's order (ss_order_of), near pairs with the regular rule, FP64.
template <bool MIXED>
__device__ __forceinline__ void sparse_entry(int64_t e, const double *__restrict__ verts,
                                             const int4 *__restrict__ tri4, const double4 *__restrict__ cen4,
                                             const double *__restrict__ area, const double4 *__restrict__ qpA, int Q,
                                             const SSTable &ss, const int32_t *__restrict__ prowptr,
                                             const int32_t *__restrict__ pcol, const int32_t *__restrict__ prow,
                                             const int32_t *__restrict__ pkind, double *__restrict__ pcorr,
                                             int64_t ld, void *__restrict__ Vout) {
  const int lane = threadIdx.x & 63;
  const int i = prow[e], j = pcol[e];
  if (j < i) return;
  const int kind = pkind[e];
  double acc = 0.0;
  double scale;
  if (kind == kNear) {
    const double4 *xa = qpA + (size_t)i * kQMax;
    const double4 *yb = qpA + (size_t)j * kQMax;
    for (int p = lane; p < Q * Q; p += 64) {
      const double4 x = xa[p / Q], y = yb[p % Q];
      const double dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
      acc += x.w * y.w * rsqrt64(dx * dx + dy * dy + dz * dz);
    }
    scale = kInv4Pi;
  } else {
    const TouchOrder o = touch_order(kind, tri4[i], tri4[j]);
    const int A = o.P[0], B = o.P[1], C = o.P[2], D0 = o.Q[0], D1 = o.Q[1], D2 = o.Q[2];
    const double ax = verts[3 * A], ay = verts[3 * A + 1], az = verts[3 * A + 2];
    const double bax = verts[3 * B] - ax, bay = verts[3 * B + 1] - ay, baz = verts[3 * B + 2] - az;
    const double cbx = verts[3 * C] - verts[3 * B], cby = verts[3 * C + 1] - verts[3 * B + 1],
                 cbz = verts[3 * C + 2] - verts[3 * B + 2];
    const double dx0 = verts[3 * D0], dy0 = verts[3 * D0 + 1], dz0 = verts[3 * D0 + 2];
    const double e1x = verts[3 * D1] - dx0, e1y = verts[3 * D1 + 1] - dy0, e1z = verts[3 * D1 + 2] - dz0;
    const double e2x = verts[3 * D2] - verts[3 * D1], e2y = verts[3 * D2 + 1] - verts[3 * D1 + 1],
                 e2z = verts[3 * D2 + 2] - verts[3 * D1 + 2];
    const double ai = area[i], aj = area[j];
    const int n = ss_order_of(ss, kind, cen4[i].w, ai, cen4[j].w, aj);
    ss_points_n(kind, ss, n, lane, [&](double x1, double x2, double y1, double y2, double wgt) {
      const double px = ax + x1 * bax + x2 * cbx, py = ay + x1 * bay + x2 * cby, pz = az + x1 * baz + x2 * cbz;
      const double qx = dx0 + y1 * e1x + y2 * e2x, qy = dy0 + y1 * e1y + y2 * e2y, qz = dz0 + y1 * e1z + y2 * e2z;
      const double rx = px - qx, ry = py - qy, rz = pz - qz;
      acc += wgt * rsqrt64(rx * rx + ry * ry + rz * rz);
    });
    scale = (2.0 * ai) * (2.0 * aj) * kInv4Pi;
  }
  const double v = wave_sum(acc) * scale;
  if (lane != 0) return;
  if (!MIXED) {
    double *V = static_cast<double *>(Vout);
    V[(size_t)i * ld + j] = v;
    V[(size_t)j * ld + i] = v;
  } else {
    float *V = static_cast<float *>(Vout);
    const float f = (float)v;
    const double corr = v - (double)f;
    V[(size_t)i * ld + j] = f;
    V[(size_t)j * ld + i] = f;
    pcorr[e] = corr;
    if (j != i) {
      // position of (j, i) in row j (columns are sorted)
      int lo = prowptr[j], hi = prowptr[j + 1] - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (pcol[mid] < i) lo = mid + 1; else hi = mid;
      }
      pcorr[lo] = corr;
    }
  }
}

// One wavefront per pattern entry.  (Fewer wavefronts taking the entries
// grid-stride were slower: an entry's chain of dependent loads is then
// waited for one entry after another.)
template <bool MIXED>
__global__ __launch_bounds__(kWG) void k_sparse(const double *__restrict__ verts, const int4 *__restrict__ tri4,
                                                const double4 *__restrict__ cen4, const double *__restrict__ area,
                                                const double4 *__restrict__ qpA, int Q, SSTable ss,
                                                const int32_t *__restrict__ prowptr, const int32_t *__restrict__ pcol,
                                                const int32_t *__restrict__ prow, const int32_t *__restrict__ pkind,
                                                double *__restrict__ pcorr, int64_t nnz, int64_t ld,
                                                void *__restrict__ Vout) {
  const int64_t e = (int64_t)blockIdx.x * (kWG / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (e < nnz)
    sparse_entry<MIXED>(e, verts, tri4, cen4, area, qpA, Q, ss, prowptr, pcol, prow, pkind, pcorr, ld, Vout);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_pad(T *V, int N, int64_t ld) {
  const int64_t pad = ld - N;
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= (int64_t)N * pad) return;
  const int64_t i = idx / pad, c = N + idx % pad;
  V[i * ld + c] = T(0);
}

// (1/4pi) (sum_k w_k / sum_k fl32(w_k))^2 for the collapsed rule of order n
static double far32_scale(int n);
// the same for the weights w[0 .. n)
static double far32_scale_w(const double *w, int n);

// Compute units of the current device (256 on MI355X), for launches sized to
// what fits on the chip at once.
static int device_cus() {
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
      hipSuccess || cus < 1)
    cus = 256;
  return cus;
}

template <int Q>
static void far_launch(bool mixed, bool low_order, const MeshView &m, int N, int64_t ld, void *V, int tiles,
                       double scale, hipStream_t s) {
  if (!mixed && !(low_order && Q == 16)) {
    hipLaunchKernelGGL((k_far64<Q, kQMax, false, 0>), dim3(tiles), dim3(kWG), 0, s, m.qpA64, m.qpS64, m.cen4, m.bbox,
                       (const int32_t *)nullptr, (const int32_t *)nullptr, N, ld, static_cast<double *>(V));
  } else if (!mixed) {
    // FP64 with Radon's rule on the tiles at least kSepFarLow64 diameters
    // apart (class 2 of bc_prepare's lists); the 4 x 4 rule on the others
    const int nt = (int)far_tiles(N);
    const int g = std::min(nt, 4 * device_cus());
    // (class 0: near, diagonal and separated non-compact tiles, differences;
    // classes 1 and 2 are separated, the expansion)
    hipLaunchKernelGGL((k_far64<16, kQMax, true, 1>), dim3(g), dim3(kWG), 0, s, m.qpA64, m.qpS64, m.cen4, m.bbox,
                       m.tile_cnt, m.tile_list, N, ld, static_cast<double *>(V));
    hipLaunchKernelGGL((k_far64<16, kQMax, true, 2>), dim3(g), dim3(kWG), 0, s, m.qpA64, m.qpS64, m.cen4, m.bbox,
                       m.tile_cnt + 1, m.tile_list + (size_t)nt, N, ld, static_cast<double *>(V));
    hipLaunchKernelGGL((k_far64<kQLow, kQLow, true, 2>), dim3(g), dim3(kWG), 0, s, m.qpLA64, m.qpLS64, m.cen4, m.bbox,
                       m.tile_cnt + 2, m.tile_list + 2 * (size_t)nt, N, ld, static_cast<double *>(V));
  } else if (Q == 16) {
    // Each tile class on its own kernel, over the tile lists of bc_prepare:
    // near and diagonal tiles on the vector ALU, separated ones on the
    // matrix cores (those at least kSepFarLow apart with Radon's rule when
    // low_order).  The matrix-core kernels run about as many workgroups as fit
    // on the chip at once and take the tiles grid-stride.
    const int cus = device_cus();
    const int nt = (int)far_tiles(N);
    const int32_t *cnt = m.tile_cnt, *list = m.tile_list;
    FarWeights w16{}, wL{};
    double x[8], w[8];
    gauss_legendre01(4, x, w);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) w16.w[4 * a + b] = (float)(w[a] * w[b] * (1.0 - x[a]));
    double rs[kQLow], rt[kQLow], rw[kQLow];
    radon7(rs, rt, rw);
    for (int a = 0; a < kQLow; ++a) wL.w[a] = (float)rw[a];
    const int gv = std::min(nt, 4 * cus), gm = std::min(nt, kFarMGrid * cus);
    hipLaunchKernelGGL((k_far32<Q, true>), dim3(gv), dim3(kWG), 0, s, m.qpA32, m.qpS32, m.cen4, m.area, cnt, list,
                       m.rsq_bias, scale, N, ld, static_cast<float *>(V));
    hipLaunchKernelGGL(k_far32m<16>, dim3(gm), dim3(kFarMWG), 0, s, m.qpA64, m.qpB16, w16, m.area, m.bbox, cnt + 1,
                       list + (size_t)nt, m.rsq_bias, scale, N, ld, static_cast<float *>(V));
    if (low_order)
      hipLaunchKernelGGL(k_far32m<kQLow>, dim3(gm), dim3(kFarMWG), 0, s, m.qpLA64, m.qpBL, wL, m.area, m.bbox,
                         cnt + 2, list + 2 * (size_t)nt, m.rsq_bias, far32_scale_w(rw, kQLow), N, ld,
                         static_cast<float *>(V));
    else
      hipLaunchKernelGGL(k_far32m<16>, dim3(gm), dim3(kFarMWG), 0, s, m.qpA64, m.qpB16, w16, m.area, m.bbox, cnt + 2,
                         list + 2 * (size_t)nt, m.rsq_bias, scale, N, ld, static_cast<float *>(V));
  } else {
    hipLaunchKernelGGL((k_far32<Q, false>), dim3(tiles), dim3(kWG), 0, s, m.qpA32, m.qpS32, m.cen4, m.area,
                       (const int32_t *)nullptr, (const int32_t *)nullptr, m.rsq_bias, scale, N, ld,
                       static_cast<float *>(V));
  }
}

// (1/4pi) (sum_k w_k / sum_k fl32(w_k))^2 for the collapsed rule of order n
static double far32_scale(int n) {
  double x[8], w[8];
  gauss_legendre01(n, x, w);
  double sw = 0.0, sf = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const double wk = w[a] * w[b] * (1.0 - x[a]);
      sw += wk;
      sf += (double)(float)wk;
    }
  return kInv4Pi * (sw / sf) * (sw / sf);
}

static double far32_scale_w(const double *w, int n) {
  double sw = 0.0, sf = 0.0;
  for (int k = 0; k < n; ++k) {
    sw += w[k];
    sf += (double)(float)w[k];
  }
  return kInv4Pi * (sw / sf) * (sw / sf);
}

int launch_assemble(const void *mesh_ws, const int32_t *tris, const double *verts, int64_t N,
                    const bc_assembly_opts &o, void *pattern, int64_t nnz, void *V, hipStream_t s) {
  (void)tris;
  const bool mixed = o.precision == BC_MIXED;
  const MeshView m = mesh_view(mesh_ws, N);
  const int64_t ld = ld_of(N);
  const int64_t T = (N + 63) / 64;
  const int tiles = (int)(T * (T + 1) / 2);
  const double scale = far32_scale(o.far_order);
  const bool low = o.far_low == 1;
  switch (o.far_order) {
    case 1: far_launch<1>(mixed, low, m, (int)N, ld, V, tiles, scale, s); break;
    case 2: far_launch<4>(mixed, low, m, (int)N, ld, V, tiles, scale, s); break;
    case 3: far_launch<9>(mixed, low, m, (int)N, ld, V, tiles, scale, s); break;
    case 4: far_launch<16>(mixed, low, m, (int)N, ld, V, tiles, scale, s); break;
    default: return BC_EINVAL;
  }
  if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  if (nnz > 0) {
    const SSTable ss = ss_table(o);
    PatternLayout P(N, nnz, o.precision);
    char *pb = static_cast<char *>(pattern);
    const int32_t *prowptr = reinterpret_cast<const int32_t *>(pb + P.rowptr);
    const int32_t *pcol = reinterpret_cast<const int32_t *>(pb + P.col);
    const int32_t *prow = reinterpret_cast<const int32_t *>(pb + P.row);
    const int32_t *pkind = reinterpret_cast<const int32_t *>(pb + P.kind);
    double *pcorr = mixed ? reinterpret_cast<double *>(pb + P.corr) : nullptr;
    const int grid = (int)((nnz + 3) / 4);
    const int Q = o.far_order * o.far_order;
    hipLaunchKernelGGL(mixed ? k_sparse<true> : k_sparse<false>, dim3(grid), dim3(kWG), 0, s, verts, m.tri4, m.cen4,
                       m.area, m.qpA64, Q, ss, prowptr, pcol, prow, pkind, pcorr, nnz, ld, V);
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  }
  if (ld > N) {
    const int64_t cnt = N * (ld - N);
    const int grid = (int)((cnt + kWG - 1) / kWG);
    if (!mixed)
      hipLaunchKernelGGL(k_pad<double>, dim3(grid), dim3(kWG), 0, s, static_cast<double *>(V), (int)N, ld);
    else
      hipLaunchKernelGGL(k_pad<float>, dim3(grid), dim3(kWG), 0, s, static_cast<float *>(V), (int)N, ld);
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  }
  return BC_OK;
}

}  // namespace bc
