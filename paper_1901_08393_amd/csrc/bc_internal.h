// Internal declarations shared by the HIP sources of libbemcap.
// Layouts of the caller-provided workspaces and the device helpers used by
// several kernels.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/bemcap.h"

namespace bc {

constexpr int kWG = 256;            // threads per workgroup (4 wave64)
constexpr int kRsqParts = 32;       // workgroups of the FP32 inverse-square-root bias (k_rsq_part)
constexpr int kQMax = 16;           // far-field points per triangle (order <= 4)
constexpr int kTileClasses = 3;     // far-field tiles: 0 near or diagonal, 1 separated, 2 distant
constexpr int kQLow = 7;            // points per triangle of the distant tiles' rule (mixed precision)
constexpr int kSSMax = 8;           // Gauss points per coordinate, singular rules
constexpr int kGMax = 256;          // workgroups per system in the solver
constexpr int kSolveWG = 1024;      // threads per solver workgroup (16 wave64)
constexpr int kNRep = 16;           // copies of the solver's release record
constexpr double kInv4Pi = 0.079577471545947667884441881686257181;  // 1/(4 pi)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int64_t ld_of(int64_t N) { return (N + 63) / 64 * 64; }

// ---------------------------------------------------------------- mesh ws
// Offsets of the tables inside the mesh workspace (all 256-byte aligned).
__host__ __device__ inline int64_t far_tiles(int64_t N) {
  const int64_t T = (N + 63) / 64;
  return T * (T + 1) / 2;
}

struct MeshLayout {
  size_t tri4, cen4, area, qpA64, qpS64, qpA32, qpS32, qpLA64, qpLS64, qpB16, qpBL, rowcnt, rowptr, kindcnt, info,
      rsqb, blockbox, tiles, total;
  explicit MeshLayout(int64_t N) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    tri4 = take(sizeof(int32_t) * 4 * N);
    cen4 = take(sizeof(double) * 4 * N);
    area = take(sizeof(double) * N);
    qpA64 = take(sizeof(double) * 4 * kQMax * N);
    qpS64 = take(sizeof(double) * 4 * kQMax * N);
    qpA32 = take(sizeof(float) * 4 * kQMax * N);
    qpS32 = take(sizeof(float) * 4 * kQMax * N);
    qpLA64 = take(sizeof(double) * 4 * kQLow * N);  // the distant tiles' rule, same layouts as qpA64 / qpS64
    qpLS64 = take(sizeof(double) * 4 * kQLow * N);
    // column operands of the matrix-core far field, per point [(b*4+c)][N]:
    // the point relative to the centre of its own 64-element block's box,
    // rounded once to FP32 (c = 0..2), and the squared norm of that FP64
    // offset rounded once (c = 3); for the 4 x 4 and the distant tiles' rule
    qpB16 = take(sizeof(float) * 4 * kQMax * N);
    qpBL = take(sizeof(float) * 4 * kQLow * N);
    rowcnt = take(sizeof(int32_t) * N);
    rowptr = take(sizeof(int32_t) * (N + 1));
    kindcnt = take(sizeof(int32_t) * 4 * N);
    info = take(sizeof(int64_t) * 8);
    // mean relative error of the FP32 hardware inverse square root, measured
    // by bc_prepare in mixed precision and divided out of every FP32 far
    // entry (one double)
    rsqb = take(sizeof(double) * (1 + kRsqParts));  // the bias, then its partial sums
    blockbox = take(sizeof(double) * 8 * ((N + 63) / 64));  // per 64 elements: min xyz, max xyz, max diam^2
    // far-field tile lists: kTileClasses counts (padded to 16), one list of
    // tile indices per class, and the per-chunk counts of the list builder
    // (chunks of 4096 tiles)
    tiles = take(sizeof(int32_t) * (16 + kTileClasses * far_tiles(N) + kTileClasses * (far_tiles(N) / 4096 + 1)));
    total = o;
  }
};

// Device view of the mesh workspace.
struct MeshView {
  const int4 *tri4;      // (v0, v1, v2, 0)
  const double4 *cen4;   // (cx, cy, cz, diam^2)
  const double *area;
  const double4 *qpA64;  // [N][Q] (x, y, z, W), rows
  const double *qpS64;   // [(b*4+c)][N], columns
  const float4 *qpA32;   // [N][Q] (x - c, y - c, z - c, W)
  const float *qpS32;    // [(b*4+c)][N]
  const int32_t *rowptr; // N + 1
  const double *bbox;    // per 64 elements: min xyz, max xyz, max diam^2, 0
  const double4 *qpLA64; // [N][kQLow], the distant tiles' rule
  const double *qpLS64;  // [(b*4+c)][N]
  const float *qpB16;    // [(b*4+c)][N], see MeshLayout
  const float *qpBL;
  const int32_t *tile_cnt;   // kTileClasses counts
  const int32_t *tile_list;  // [kTileClasses][far_tiles(N)]
  const double *rsq_bias;    // see MeshLayout::rsqb
};

inline MeshView mesh_view(const void *ws, int64_t N) {
  MeshLayout L(N);
  const char *b = static_cast<const char *>(ws);
  MeshView v;
  v.tri4 = reinterpret_cast<const int4 *>(b + L.tri4);
  v.cen4 = reinterpret_cast<const double4 *>(b + L.cen4);
  v.area = reinterpret_cast<const double *>(b + L.area);
  v.qpA64 = reinterpret_cast<const double4 *>(b + L.qpA64);
  v.qpS64 = reinterpret_cast<const double *>(b + L.qpS64);
  v.qpA32 = reinterpret_cast<const float4 *>(b + L.qpA32);
  v.qpS32 = reinterpret_cast<const float *>(b + L.qpS32);
  v.rowptr = reinterpret_cast<const int32_t *>(b + L.rowptr);
  v.bbox = reinterpret_cast<const double *>(b + L.blockbox);
  v.qpLA64 = reinterpret_cast<const double4 *>(b + L.qpLA64);
  v.qpLS64 = reinterpret_cast<const double *>(b + L.qpLS64);
  v.qpB16 = reinterpret_cast<const float *>(b + L.qpB16);
  v.qpBL = reinterpret_cast<const float *>(b + L.qpBL);
  v.tile_cnt = reinterpret_cast<const int32_t *>(b + L.tiles);
  v.tile_list = v.tile_cnt + 16;
  v.rsq_bias = reinterpret_cast<const double *>(b + L.rsqb);
  return v;
}

// ------------------------------------------------------------- pattern ws
enum PairKind : int32_t { kNear = 0, kVertex = 1, kEdge = 2, kCoincident = 3 };

struct PatternLayout {
  size_t rowptr, col, row, kind, corr, total;
  PatternLayout(int64_t N, int64_t nnz, int32_t precision) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    rowptr = take(sizeof(int32_t) * (N + 1));
    col = take(sizeof(int32_t) * nnz);
    row = take(sizeof(int32_t) * nnz);
    kind = take(sizeof(int32_t) * nnz);
    corr = precision == BC_MIXED ? take(sizeof(double) * nnz) : o;
    total = o;
  }
};

// ---------------------------------------------------------------- solver ws
// Barrier slot of one solver workgroup (its partial sums and arrival tag)
// and the release record the master workgroup publishes; 64 bytes each.
struct alignas(64) BarSlot {
  double v[4];
  unsigned tag;
  unsigned pad[7];
};
struct alignas(64) BarRel {
  double v[4];
  unsigned gen;
  int abort;
  unsigned pad[6];
};

// Symmetric product.  V is read only on its diagonal blocks and above them:
// rows are grouped in blocks of kRB, and block b is swept from column kRB*b to
// ld.  With several vectors (the dual mesh's products) the sweep is cut into
// chunks of 64*k columns (k entries per lane); a unit is one (block, chunk)
// pair, units are numbered block by block and the workgroups of a system take
// equal contiguous ranges of them.  With one vector it is cut into strips
// (below).
constexpr int kRB = 128;        // rows per block of the symmetric product
constexpr int kMaxBand = 1536;  // rows of the vectors owned by one solver workgroup

// Units of the blocks 0..B-1, m64 = ld / 64.  Block b has
// ceil((m64 - 2b) / k) units; the sum is written out for k = 1, 2 and 4
// (pairs of blocks for k = 4; only k = 1 is in use).
__host__ __device__ inline int64_t half_units_before(int64_t B, int64_t m64, int k) {
  if (k == 1) return B * m64 - B * (B - 1);
  if (k == 2) return B * ((m64 + 1) / 2) - B * (B - 1) / 2;
  const int64_t n = m64 + 3, f0 = n / 4, f2 = (n - 2) / 4, A = B / 2;
  int64_t s = A * (f0 + f2) - A * (A - 1);
  if (B & 1) s += f0 - A;
  return s;
}

// Strip sweep of the symmetric product with one vector: block b is swept
// from column kRB*b to ld in strips of 256 bytes of each row (64 FP32 or 32
// FP64 columns, a divisor of 64), and the wavefronts of a system take equal
// contiguous ranges of the strips, numbered block by block.  Block b has
// (ld - kRB b) / sw strips.
constexpr int kStripBytes = 256;
__host__ __device__ inline int64_t strips_before(int64_t B, int64_t ld, int sw) {
  return B * (ld / sw) - (kRB / sw) * (B * (B - 1) / 2);
}
// Workgroups of one system in the solver: about 80 rows (5 per wavefront)
// each, at most kGMax.
__host__ __device__ inline int solve_wg_count(int64_t N) {
  int64_t g = (N + 79) / 80;
  if (g < 1) g = 1;
  if (g > kGMax) g = kGMax;
  return (int)g;
}
// Row-sum slots of a strip sweep: the segment of wavefront g (of GH) in row
// block B is stored at slot g + B, which no other segment shares (a later
// wavefront never holds an earlier block).
__host__ __device__ inline int64_t strip_slots(int64_t N) {
  return 16 * (int64_t)solve_wg_count(N) + (N + kRB - 1) / kRB;
}

// Offsets inside one system's solver workspace (256-byte aligned).
//   ctl    control block, then the solver descriptor of bc_solve
//   slots  barrier slots, one per workgroup;  rel  release records
//   x64 r64   FP64 iterate and residual
//   vec    r u w p s d invdiag in the matrix precision
//   rpart  row partial sums of the symmetric product, kRB per slot
//   cpart  column partial sums, ld per row block
struct SolveLayout {
  size_t ctl, slots, rel, x64, r64, vec, rpart, cpart, total;
  int64_t ld, nB, T;
  int sw;  // strip width in columns
  __host__ __device__ SolveLayout(int64_t N, int32_t precision) {
    ld = (N + 63) / 64 * 64;
    sw = kStripBytes / (precision == BC_FP64 ? 8 : 4);
    nB = (N + kRB - 1) / kRB;
    T = strips_before(nB, ld, sw);
    size_t o = 0;
    auto take = [&](size_t bytes) {
      size_t r = o;
      o = (o + bytes + 255) & ~size_t(255);
      return r;
    };
    ctl = take(1024);
    slots = take(sizeof(BarSlot) * kGMax);
    rel = take(sizeof(BarRel) * kNRep);
    x64 = take(sizeof(double) * ld);
    r64 = take(sizeof(double) * ld);
    vec = take((precision == BC_FP64 ? 8 : 4) * ld * 7);
    // FP64 row sums (those of the residual product in mixed precision)
    rpart = take(sizeof(double) * kRB * (size_t)strip_slots(N));
    cpart = take(sizeof(double) * (size_t)ld * (size_t)nB);
    total = o;
  }
};

// Product kind of an FP32 matrix with FP64 vectors.
constexpr int32_t kMatvecF32X64 = BC_F32_F64;

// Workspace of a standalone product y = V x (bc_matvec): x padded to ld
// with zeros, then the partial sums of the symmetric product.
struct MatvecLayout {
  size_t xpad, rpart, cpart, total;
  int64_t ld, nB, T;
  int k;   // several vectors: unit width / 64 (one column per lane)
  int sw;  // one vector: strip width in columns
  // kind: BC_FP64, BC_MIXED (FP32 matrix and vectors) or kMatvecF32X64
  // (FP32 matrix, FP64 vectors).  One vector: the strip sweep (row sums per
  // slot); several: units of kRB rows x 64 columns swept by workgroups (row
  // sums per unit).
  __host__ __device__ MatvecLayout(int64_t N, int32_t kind, int nr = 1) {
    ld = (N + 63) / 64 * 64;
    k = 1;
    sw = kStripBytes / (kind == BC_FP64 ? 8 : 4);
    nB = (N + kRB - 1) / kRB;
    T = nr > 1 ? half_units_before(nB, ld / 64, k) : strips_before(nB, ld, sw);
    size_t o = 0;
    auto take = [&](size_t bytes) {
      size_t r = o;
      o = (o + bytes + 255) & ~size_t(255);
      return r;
    };
    xpad = take(sizeof(double) * (size_t)nr * (size_t)ld);
    rpart = take(sizeof(double) * (size_t)nr * kRB * (size_t)(nr > 1 ? T : strip_slots(N)));
    cpart = take(sizeof(double) * (size_t)nr * (size_t)ld * (size_t)nB);
    total = o;
  }
};

// Workspace of the dual-mesh system (bc_dual_*).
struct DualLayout {
  size_t area, diam, curl, f, mdiag, basis, wbas, ubas, w, t1, t2, t3, eta2, ones, bvec, yvec, dots, mv, gctl, H, G,
      rot, total;
  int64_t nb;
  DualLayout(int64_t N, int64_t M, int32_t restart);
};

// Per-system control block at the start of the solver workspace.  Written
// only by workgroup 0 of the system (state save) and by the barrier.
struct SolveCtl {
  unsigned bar_count;  // unused (kept for layout stability)
  unsigned bar_gen;    // unused
  int32_t abort;       // unused
  int32_t phase;
  int32_t iters;
  int32_t outer;
  int32_t inner;
  int32_t status;
  uint32_t epoch;
  int32_t hs_n;  // terms alpha_j gamma_j of the current inner solve so far
  double bnorm, rnorm, scale, gamma, eta, alpha, beta, itol;
  // capacity stop (cap_rtol > 0): the last four terms alpha_j gamma_j of the
  // current inner solve, their running sum, the functional J = b^T x + x^T r
  // at its start, the scale rnorm^2 of its terms, and the estimate of the
  // capacity's algebraic error (J units) it ended with (< 0: none)
  double hs[4], hs_sum, jres, est;
};

// Solver descriptor built by the host for each system of a launch.
struct SysDesc {
  const void *V;
  const int32_t *prowptr;
  const int32_t *pcol;
  const double *pcorr;
  const double *area;
  double *sigma;
  char *ws;
  bc_result *result;
  int64_t N;
  int64_t ld;
  int64_t nnz;
  int32_t wg_begin;
  int32_t wg_count;
  int32_t start;
  int32_t budget;  // > 0: this system's product bound in this launch
};

struct SolveParams {
  double rtol, inner_rtol, cap_rtol;
  int32_t max_iter, max_outer, jacobi, x0_given;
  int32_t iter_budget;
  uint32_t spin_limit;
  int32_t n_sys;
};

// --------------------------------------------------------- device helpers
// Pointers in the global address space.  Pointers read from descriptors in
// memory are generic to the compiler, which would then emit flat loads;
// casting them once makes every access a global load/store.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;
template <typename T>
using lptr = T __attribute__((address_space(3))) *;  // LDS
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T *p) {
  return (gptr<T>)p;
}

// Inverse square root in FP64: hardware estimate refined by one step of the
// cubically convergent iteration y <- y (1 + e/2 + 3e^2/8), e = 1 - x y^2
// (Householder's method of order 2 applied to f(y) = y^-2 - x).
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double t = x * y;
  double e = __builtin_fma(-t, y, 1.0);
  double c = __builtin_fma(0.375, e, 0.5);
  return __builtin_fma(y * e, c, y);
}

// Squared distance between two axis-aligned boxes given as (min xyz, max
// xyz); 0 if they touch or overlap.
__device__ __forceinline__ double box_dist2(const double *a, const double *b) {
  double s = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double g = fmax(0.0, fmax(a[c] - b[3 + c], b[c] - a[3 + c]));
    s += g * g;
  }
  return s;
}

// Far-field tiles: 64 x 64 element pairs (I, J) of the upper block
// triangle, enumerated column-block first: t = J (J + 1) / 2 + I, I <= J.
__device__ __forceinline__ void tile_of(int t, int &I, int &J) {
  int j = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  while (j * (j + 1) / 2 > t) --j;
  J = j;
  I = t - j * (j + 1) / 2;
}

// Tiles whose 64-element blocks' bounding boxes are at least kSepFar
// largest element diameters apart use the expanded distance form in the
// far-field kernels (on the matrix cores in FP32).
constexpr double kSepFar = 4.0;

__device__ __forceinline__ bool far_separated(const double *bbox, int I, int J) {
  const double *bi = bbox + 8 * I, *bj = bbox + 8 * J;
  return box_dist2(bi, bj) >= kSepFar * kSepFar * fmax(bi[6], bj[6]);
}

// Tiles at least kSepFarLow largest element diameters apart may take, in
// mixed precision, Radon's 7-point rule of degree 5 on each triangle (49
// point pairs instead of 256).  For triangle pairs at centroid distance
// d >= 8 diameters its relative error against a high-order rule is at most
// 6e-10 (mean 1e-10) over random shapes and orientations, falling as d^-6;
// the FP32 rounding of the stored entry is 6e-8.
constexpr double kSepFarLow = 8.0;
// In FP64 the same rule is taken from 32 diameters, where its relative
// error is at most 1.4e-13 (the FP64 entries stay within 2e-13 of those of
// the 4 x 4 rule; at 24 diameters 6.6e-13, at 16 9e-12).
constexpr double kSepFarLow64 = 32.0;

__device__ __forceinline__ bool far_low_order(const double *bbox, int I, int J, double sep = kSepFarLow) {
  const double *bi = bbox + 8 * I, *bj = bbox + 8 * J;
  return box_dist2(bi, bj) >= sep * sep * fmax(bi[6], bj[6]);
}

// Gauss rules of the singular quadrature for every order a launch may use
// (row n: the n-point rule on [0, 1]) and how a touching pair picks its
// order: `base` for coincident pairs, `edge` / `vertex` for edge- and
// vertex-adjacent pairs (0: base), raised to `sliver` when an element of
// the pair has diam^2 > sliver_ratio |T| (sliver 0: off).
struct SSTable {
  double x[kSSMax + 1][kSSMax], w[kSSMax + 1][kSSMax];
  int32_t base, edge, vertex, sliver;
  double sliver_ratio;
};

// filled from the assembly options on the host (abi.hip)
SSTable ss_table(const bc_assembly_opts &o);

__device__ __forceinline__ int ss_order_of(const SSTable &t, int kind, double d2i, double ai, double d2j,
                                           double aj) {
  int n = t.base;
  if (kind == kEdge && t.edge > 0) n = t.edge;
  else if (kind == kVertex && t.vertex > 0) n = t.vertex;
  if (t.sliver > 0 && (d2i > t.sliver_ratio * ai || d2j > t.sliver_ratio * aj)) n = max(n, t.sliver);
  return n;
}

// Region maps of the singular rules on K = {0 <= x2 <= x1 <= 1}; (xi, e1,
// e2, e3) in [0,1]^4.  Returns the Jacobian and writes the two reference
// points.  kind: 3 coincident (6 regions), 2 edge (4), 1 vertex (2).
__device__ __forceinline__ double ss_map(int kind, int reg, double xi, double e1, double e2, double e3, double &x1,
                                         double &x2, double &y1, double &y2) {
  double a1, a2, b1, b2, J;
  if (kind == kCoincident) {
    J = xi * xi * xi * e1 * e1 * e2;
    int r = reg >> 1;
    if (r == 0) {
      a1 = xi; a2 = xi * (1.0 - e1 + e1 * e2);
      b1 = xi * (1.0 - e1 * e2 * e3); b2 = xi * (1.0 - e1);
    } else if (r == 1) {
      a1 = xi; a2 = xi * e1 * (1.0 - e2 + e2 * e3);
      b1 = xi * (1.0 - e1 * e2); b2 = xi * e1 * (1.0 - e2);
    } else {
      a1 = xi * (1.0 - e1 * e2 * e3); a2 = xi * e1 * (1.0 - e2 * e3);
      b1 = xi; b2 = xi * e1 * (1.0 - e2);
    }
  } else if (kind == kEdge) {
    if ((reg & 1) == 0) {   // {p >= w + r}
      J = xi * xi * xi * e1 * e1 * e2;
      a1 = xi; a2 = xi * e1;
      b1 = xi * (1.0 - e1 * e2 * e3); b2 = xi * e1 * e2 * (1.0 - e3);
    } else {                // {p <= w + r}
      J = xi * xi * xi * e1 * e1;
      a1 = xi; a2 = xi * e1 * e3;
      b1 = xi * (1.0 - e1 * e2); b2 = xi * e1 * (1.0 - e2);
    }
  } else {
    J = xi * xi * xi * e2;
    a1 = xi; a2 = xi * e1;
    b1 = xi * e2; b2 = xi * e2 * e3;
  }
  // odd regions are the mirror images (the two triangles swap roles)
  if (kind == kEdge) {
    // edge regions are ordered A, B, mirror A, mirror B
    if (reg >= 2) { double t1 = a1, t2 = a2; a1 = b1; a2 = b2; b1 = t1; b2 = t2; }
  } else if (reg & 1) {
    double t1 = a1, t2 = a2; a1 = b1; a2 = b2; b1 = t1; b2 = t2;
  }
  x1 = a1; x2 = a2; y1 = b1; y2 = b2;
  return J;
}

// The points of the singular rule of order n for a pair of class `kind`,
// shared out over the 64 lanes of a wavefront: f(x1, x2, y1, y2, w) per
// point, with the reference points of both triangles and the weight (the
// Jacobian included).  NSS > 0 makes the order a compile-time constant, so
// that the point index splits into Gauss indices by shifts.
template <int NSS, typename F>
__device__ __forceinline__ void ss_points(int kind, const double *sx, const double *sw, int nrt, int lane, F &&f) {
  const int n = NSS > 0 ? NSS : nrt, n2 = n * n, n4 = n2 * n2;
  const int nreg = kind == kCoincident ? 6 : (kind == kEdge ? 4 : 2);
  for (int p = lane; p < nreg * n4; p += 64) {
    const int reg = p / n4;
    int q = p - reg * n4;
    const int i3 = q % n; q /= n;
    const int i2 = q % n; q /= n;
    const int i1 = q % n; q /= n;
    const int i0 = q;
    double x1, x2, y1, y2;
    const double Jac = ss_map(kind, reg, sx[i0], sx[i1], sx[i2], sx[i3], x1, x2, y1, y2);
    f(x1, x2, y1, y2, sw[i0] * sw[i1] * sw[i2] * sw[i3] * Jac);
  }
}

// ss_points for the pair's order n (uniform in the wavefront): orders 4
// and 8 compiled as constants, the others at run time.
template <typename F>
__device__ __forceinline__ void ss_points_n(int kind, const SSTable &t, int n, int lane, F &&f) {
  if (n == 4) ss_points<4>(kind, t.x[4], t.w[4], 4, lane, f);
  else if (n == 8) ss_points<8>(kind, t.x[8], t.w[8], 8, lane, f);
  else ss_points<0>(kind, t.x[n], t.w[n], n, lane, f);
}

// Canonical vertex orders of a touching pair, the first element p and the
// second q, as the singular rules use them: P = (A, B, C) on T_p and
// Q = (D0, D1, D2) on T_q.
//   coincident: P = Q = T_p in input order;
//   edge:       {A, B} the shared edge, A the lower vertex index, C the free
//               vertex of T_p; Q = (A, B, D), D the free vertex of T_q;
//   vertex:     A the shared vertex, B and C the other vertices of T_p in its
//               cyclic input order after A; Q = (A, D, E) likewise for T_q.
// sp[c], sq[c]: the input slot (0..2) of P[c] in T_p and of Q[c] in T_q.
struct TouchOrder {
  int P[3], Q[3], sp[3], sq[3];
};

__device__ __forceinline__ TouchOrder touch_order(int kind, int4 tp, int4 tq) {
  const int tv[3] = {tp.x, tp.y, tp.z}, sv[3] = {tq.x, tq.y, tq.z};
  TouchOrder o;
  if (kind == kCoincident) {
    for (int c = 0; c < 3; ++c) { o.P[c] = tv[c]; o.Q[c] = tv[c]; }
  } else if (kind == kEdge) {
    int sh[2] = {0, 0}, ns = 0, c = -1, d = -1;
    for (int a = 0; a < 3; ++a) {
      const bool in = tv[a] == sv[0] || tv[a] == sv[1] || tv[a] == sv[2];
      if (in) sh[ns++ & 1] = tv[a]; else c = tv[a];
      const bool jn = sv[a] == tv[0] || sv[a] == tv[1] || sv[a] == tv[2];
      if (!jn) d = sv[a];
    }
    o.P[0] = min(sh[0], sh[1]); o.P[1] = max(sh[0], sh[1]); o.P[2] = c;
    o.Q[0] = o.P[0]; o.Q[1] = o.P[1]; o.Q[2] = d;
  } else {
    int ki = 0, kj = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (tv[a] == sv[b]) { ki = a; kj = b; }
    o.P[0] = tv[ki]; o.P[1] = tv[(ki + 1) % 3]; o.P[2] = tv[(ki + 2) % 3];
    o.Q[0] = o.P[0]; o.Q[1] = sv[(kj + 1) % 3]; o.Q[2] = sv[(kj + 2) % 3];
  }
  for (int c = 0; c < 3; ++c) {
    o.sp[c] = o.P[c] == tv[0] ? 0 : (o.P[c] == tv[1] ? 1 : 2);
    o.sq[c] = o.Q[c] == sv[0] ? 0 : (o.Q[c] == sv[1] ? 1 : 2);
  }
  return o;
}

// The matrix-core far field expands -r^2 = 2 e.y - |e|^2 - |y|^2 about the
// centre of the column block's box, so its FP32 rounding error grows like
// (|e|^2 + |y|^2) / r^2.  A tile takes that kernel only if the column block
// is compact against the gap: the half-diagonal of its box at most
// kCompact times the box distance.  Blocks of spatially scattered elements
// (a caller's element order) fail the test and keep the vector-ALU kernel,
// which expands about each column element's own centroid.
constexpr double kCompact = 2.5;

__device__ __forceinline__ bool far_compact(const double *bbox, int I, int J) {
  const double *bj = bbox + 8 * J;
  double h2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double d = 0.5 * (bj[3 + c] - bj[c]);
    h2 += d * d;
  }
  return h2 <= kCompact * kCompact * box_dist2(bbox + 8 * I, bj);
}

// Fused multiply-add in the type of the operands (__builtin_fma alone would
// promote float operands to double).
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Sum over the 64 lanes of a wavefront with a fixed butterfly order; every
// lane receives the total.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 64 lanes of a wavefront whose lanes are all active, with
// DPP lane exchanges (fixed order): pairs and quads by quad permutations,
// eight and sixteen lanes by the half-row and row mirrors, then the four
// rows of sixteen read out in order, ((r0 + r1) + (r2 + r3)).  Needs no lane
// index and no LDS; every lane receives the total.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_f(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename T>
__device__ __forceinline__ T wave_sum_full(T v) {
  v += dpp_f<0xB1>(v);   // quad_perm(1,0,3,2): lane ^ 1
  v += dpp_f<0x4E>(v);   // quad_perm(2,3,0,1): lane ^ 2
  v += dpp_f<0x141>(v);  // row_half_mirror: the other quad of eight
  v += dpp_f<0x140>(v);  // row_mirror: the other eight of sixteen
  return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}

}  // namespace bc

// Host-side launchers (each returns a bc_status).
namespace bc {
int launch_geometry(const double *verts, const int32_t *tris, int64_t N, int far_order, void *mesh_ws,
                    hipStream_t s);
// the mean error of the FP32 hardware inverse square root into the mesh
// workspace (MeshLayout::rsqb)
int launch_rsq_bias(void *mesh_ws, int64_t N, hipStream_t s);
int launch_pattern(const double *verts, const int32_t *tris, int64_t N, double near_factor, const void *mesh_ws,
                   void *pattern, int64_t nnz, int32_t precision, bool emit, hipStream_t s);
int launch_assemble(const void *mesh_ws, const int32_t *tris, const double *verts, int64_t N,
                    const bc_assembly_opts &o, void *pattern, int64_t nnz, void *V, hipStream_t s);
// weighted-residual estimator: workspace bytes and the three kernels
size_t residual_workspace_bytes(int64_t N, int64_t nnz);
int launch_residual(const double *verts, int64_t N, const bc_assembly_opts &o, const void *mesh_ws,
                    const void *pattern, int64_t nnz, const double *sigma, double *mu2, double *mom, void *ws,
                    hipStream_t s);
int launch_zz(const int32_t *tris, int64_t N, const void *mesh_ws, const void *pattern, int64_t nnz,
              const double *sigma, int h_mode, double *eta2, hipStream_t s);
int launch_capacity(const double *sigma, const double *area, int64_t N, double *cap, hipStream_t s);
int launch_solve(int32_t precision, const SysDesc *d_desc, int n_sys, int total_wg, const SolveParams &p,
                 hipStream_t s);
int solve_capacity(int32_t precision);
// Y = V X for nr vectors stored one after the other (N entries each): kind
// BC_FP64 with nr = 1 or 3, BC_MIXED (FP32 matrix and vectors) with nr = 1,
// kMatvecF32X64 (FP32 matrix, FP64 vectors and sums) with nr = 1 or 3.
// ws: MatvecLayout(N, kind, nr).
// skip (may be NULL): a device flag; the launches do nothing while it is set.
int launch_matvec(int32_t kind, const void *V, int64_t N, int nr, const void *x, void *y, void *ws, hipStream_t s,
                  const int32_t *skip = nullptr);
int launch_dual_setup(const double *verts, const int32_t *tris, int64_t N, int64_t M, const int32_t *iptr,
                      const int32_t *itri, void *ws, int32_t restart, hipStream_t s);
// V_bary: FP64 (precision BC_FP64) or FP32 plus the FP64 correction of the
// pattern's entries (BC_MIXED; pattern = the bc_assemble pattern buffer).
int run_dual_solve(const void *Vb, int32_t precision, const void *pattern, int64_t nnz, const int32_t *tris, int64_t N,
                   int64_t M, const int32_t *iptr, const int32_t *itri, const int32_t *icor, void *ws,
                   const bc_dual_opts &o, double *x, bc_dual_result *res, hipStream_t s);
int launch_dual_zz(const void *ws, const int32_t *tris, int64_t N, int64_t M, int32_t restart, const double *x,
                   int h_mode, double *eta2, hipStream_t s);
int solve_workgroups(int64_t N);
// bc_solve on the workspace d_ws (ws_bytes long)
int solve_one(const void *d_V, int64_t N, int32_t precision, const void *d_pattern, int64_t nnz, const double *d_area,
              double *d_sigma, const bc_solve_opts *opts, void *d_ws, size_t ws_bytes, bc_result *d_result,
              hipStream_t s);
int launch_set_desc(const SysDesc *h, int n, SysDesc *d, hipStream_t s);
void gauss_legendre01(int n, double *x, double *w);
void radon7(double *s, double *t, double *w);
}  // namespace bc
