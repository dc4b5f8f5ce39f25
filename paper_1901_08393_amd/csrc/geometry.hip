// Element geometry, far-field quadrature tables and pair classification.
//
// Geometry (Section 2.1, plane triangles): area, centroid, squared diameter,
// and the points/weights of the collapsed Gauss rule on each triangle, in
// two layouts: per element (rows of the far-field kernel read one element's
// points with uniform loads) and per point (columns read one point of 64
// consecutive elements with coalesced loads).  FP32 copies are stored
// relative to the element centroid so that differences of nearby points do
// not cancel in FP32, with the reference-triangle weight in place of 2|T| w.
//
// Classification (pairs are told apart by shared vertex indices of the
// conforming mesh, Section 2.1): for every ordered pair (i, j) the number of
// shared vertices decides coincident / edge / vertex; pairs sharing none are
// "near" when |c_i - c_j|^2 < nf^2 max(diam_i^2, diam_j^2).  The pattern is
// built in two passes (count, then emit at scanned offsets) so that entries
// are in (row, column) order without atomics.
#include "bc_internal.h"

namespace bc {

struct FarRule {
  int Q;
  int pad;
  double s[kQMax], t[kQMax], w[kQMax];
};

__global__ __launch_bounds__(kWG) void k_geometry(const double *__restrict__ verts,
                                                  const int32_t *__restrict__ tris, int N, FarRule rule,
                                                  FarRule ruleL, int4 *tri4, double4 *cen4, double *area,
                                                  double4 *qpA64, double *qpS64, float4 *qpA32, float *qpS32,
                                                  double4 *qpLA64, double *qpLS64) {
#pragma clang fp contract(off)
  int e = blockIdx.x * kWG + threadIdx.x;
  if (e >= N) return;
  int a = tris[3 * e], b = tris[3 * e + 1], c = tris[3 * e + 2];
  double p0x = verts[3 * a], p0y = verts[3 * a + 1], p0z = verts[3 * a + 2];
  double p1x = verts[3 * b], p1y = verts[3 * b + 1], p1z = verts[3 * b + 2];
  double p2x = verts[3 * c], p2y = verts[3 * c + 1], p2z = verts[3 * c + 2];
  double ux = p1x - p0x, uy = p1y - p0y, uz = p1z - p0z;
  double vx = p2x - p0x, vy = p2y - p0y, vz = p2z - p0z;
  double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  double A = 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
  double cx = (p0x + p1x + p2x) / 3.0, cy = (p0y + p1y + p2y) / 3.0, cz = (p0z + p1z + p2z) / 3.0;
  double d01x = p1x - p0x, d01y = p1y - p0y, d01z = p1z - p0z;
  double d12x = p2x - p1x, d12y = p2y - p1y, d12z = p2z - p1z;
  double d20x = p0x - p2x, d20y = p0y - p2y, d20z = p0z - p2z;
  double l01 = d01x * d01x + d01y * d01y + d01z * d01z;
  double l12 = d12x * d12x + d12y * d12y + d12z * d12z;
  double l20 = d20x * d20x + d20y * d20y + d20z * d20z;
  double diam2 = fmax(fmax(l01, l12), l20);
  tri4[e] = make_int4(a, b, c, 0);
  cen4[e] = make_double4(cx, cy, cz, diam2);
  area[e] = A;
  for (int k = 0; k < kQMax; ++k) {
    double x = 0, y = 0, z = 0, W = 0;
    if (k < rule.Q) {
      x = p0x + rule.s[k] * ux + rule.t[k] * vx;
      y = p0y + rule.s[k] * uy + rule.t[k] * vy;
      z = p0z + rule.s[k] * uz + rule.t[k] * vz;
      W = 2.0 * A * rule.w[k];
    }
    qpA64[(size_t)e * kQMax + k] = make_double4(x, y, z, W);
    qpS64[(size_t)(k * 4 + 0) * N + e] = x;
    qpS64[(size_t)(k * 4 + 1) * N + e] = y;
    qpS64[(size_t)(k * 4 + 2) * N + e] = z;
    qpS64[(size_t)(k * 4 + 3) * N + e] = W;
    float rx = k < rule.Q ? (float)(x - cx) : 0.f;
    float ry = k < rule.Q ? (float)(y - cy) : 0.f;
    float rz = k < rule.Q ? (float)(z - cz) : 0.f;
    // FP32 tables carry the reference weight only; the element areas are
    // applied per entry in FP64 (see k_far32)
    float rw = k < rule.Q ? (float)rule.w[k] : 0.f;
    qpA32[(size_t)e * kQMax + k] = make_float4(rx, ry, rz, rw);
    qpS32[(size_t)(k * 4 + 0) * N + e] = rx;
    qpS32[(size_t)(k * 4 + 1) * N + e] = ry;
    qpS32[(size_t)(k * 4 + 2) * N + e] = rz;
    qpS32[(size_t)(k * 4 + 3) * N + e] = rw;
  }
  // the rule of the distant tiles in mixed precision
  for (int k = 0; k < kQLow; ++k) {
    const double x = p0x + ruleL.s[k] * ux + ruleL.t[k] * vx;
    const double y = p0y + ruleL.s[k] * uy + ruleL.t[k] * vy;
    const double z = p0z + ruleL.s[k] * uz + ruleL.t[k] * vz;
    const double W = 2.0 * A * ruleL.w[k];
    qpLA64[(size_t)e * kQLow + k] = make_double4(x, y, z, W);
    qpLS64[(size_t)(k * 4 + 0) * N + e] = x;
    qpLS64[(size_t)(k * 4 + 1) * N + e] = y;
    qpLS64[(size_t)(k * 4 + 2) * N + e] = z;
    qpLS64[(size_t)(k * 4 + 3) * N + e] = W;
  }
}

// Shared vertices of two triangles (0..3).
__device__ __forceinline__ int shared_count(int a0, int a1, int a2, int b0, int b1, int b2) {
  return (a0 == b0) + (a0 == b1) + (a0 == b2) + (a1 == b0) + (a1 == b1) + (a1 == b2) + (a2 == b0) +
         (a2 == b1) + (a2 == b2);
}

// Pair class of (i, j): 3/2/1 = coincident/edge/vertex, 0 = near, -1 = none.
// The distance test is written without contraction so that it rounds like
// the plain expression ((dx dx + dy dy) + dz dz) < nf2 max(d2_i, d2_j).
__device__ __forceinline__ int pair_class(int4 ti, double4 ci, int4 tj, double4 cj, double nf2) {
#pragma clang fp contract(off)
  int s = shared_count(ti.x, ti.y, ti.z, tj.x, tj.y, tj.z);
  if (s > 0) return s;
  if (nf2 > 0.0) {
    double dx = ci.x - cj.x, dy = ci.y - cj.y, dz = ci.z - cj.z;
    double r2 = dx * dx + dy * dy + dz * dz;
    double thr = nf2 * fmax(ci.w, cj.w);
    if (r2 < thr) return kNear;
  }
  return -1;
}

// Axis-aligned box of the vertices of each block of 64 consecutive elements
// and the largest squared diameter in the block: one wavefront per block.
__global__ __launch_bounds__(64) void k_blockbox(const double *__restrict__ verts, const int4 *__restrict__ tri4,
                                                 const double4 *__restrict__ cen4, int N, double *box) {
  const int B = blockIdx.x, lane = threadIdx.x;
  const int e = min(B * 64 + lane, N - 1);
  const int4 t = tri4[e];
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) {
    const double a = verts[3 * t.x + c], b = verts[3 * t.y + c], d = verts[3 * t.z + c];
    lo[c] = fmin(fmin(a, b), d);
    hi[c] = fmax(fmax(a, b), d);
  }
  double d2 = cen4[e].w;
  for (int off = 32; off >= 1; off >>= 1) {
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], __shfl_xor(lo[c], off, 64));
      hi[c] = fmax(hi[c], __shfl_xor(hi[c], off, 64));
    }
    d2 = fmax(d2, __shfl_xor(d2, off, 64));
  }
  if (lane == 0) {
    double *o = box + 8 * B;
    o[0] = lo[0]; o[1] = lo[1]; o[2] = lo[2];
    o[3] = hi[0]; o[4] = hi[1]; o[5] = hi[2];
    o[6] = d2; o[7] = 0.0;
  }
}


// Column operands of the matrix-core far field (MeshLayout::qpB16, qpBL):
// each point of the 4 x 4 and the distant tiles' rules relative to the centre of its own
// element block's box (FP64, rounded once) and the squared norm of that
// offset.  The kernel takes the frame of the column block, which is the
// column element's own block, so these are per element.
__global__ __launch_bounds__(kWG) void k_colpoints(const double *__restrict__ qpS64, const double *__restrict__ qpLS64,
                                                   const double *__restrict__ bbox, int N, float *__restrict__ qpB16,
                                                   float *__restrict__ qpBL) {
  const int e = blockIdx.x * kWG + threadIdx.x;
  if (e >= N) return;
  const double *bx = bbox + 8 * (e / 64);
  const double fx = 0.5 * (bx[0] + bx[3]), fy = 0.5 * (bx[1] + bx[4]), fz = 0.5 * (bx[2] + bx[5]);
  auto put = [&](const double *S, float *B, int nq) {
    for (int b = 0; b < nq; ++b) {
      const double yx = S[(size_t)(b * 4 + 0) * N + e] - fx;
      const double yy = S[(size_t)(b * 4 + 1) * N + e] - fy;
      const double yz = S[(size_t)(b * 4 + 2) * N + e] - fz;
      B[(size_t)(b * 4 + 0) * N + e] = (float)yx;
      B[(size_t)(b * 4 + 1) * N + e] = (float)yy;
      B[(size_t)(b * 4 + 2) * N + e] = (float)yz;
      B[(size_t)(b * 4 + 3) * N + e] = (float)(yx * yx + yy * yy + yz * yz);
    }
  };
  put(qpS64, qpB16, kQMax);
  put(qpLS64, qpBL, kQLow);
}

// Far-field tile lists: the tiles of the upper block triangle of each class
// (kTileClasses), in tile order, so that each far-field kernel runs over its
// own tiles only and neighbouring workgroups share column blocks in the
// cache.  Two passes over chunks of kTileChunk tiles: counts per chunk, then
// each chunk's offsets (the counts of the chunks before it) and its tiles'
// ranks (a scan over the workgroup's threads, 16 consecutive tiles each).
constexpr int kTilesPerThread = 16;
constexpr int kTileChunk = kWG * kTilesPerThread;
static_assert(kTileChunk == 4096, "MeshLayout sizes the per-chunk counts for chunks of 4096 tiles");

// Far-field tile classes: 0 near or diagonal (or a column block that is not
// compact against the gap), 1 separated, 2 distant (Radon's rule: from
// kSepFarLow diameters in mixed precision, kSepFarLow64 in FP64).
__device__ __forceinline__ int tile_class(const double *bbox, int t, double sep_low) {
  int I, J;
  tile_of(t, I, J);
  return (I == J || !far_separated(bbox, I, J) || !far_compact(bbox, I, J)) ? 0
                                                                            : (far_low_order(bbox, I, J, sep_low) ? 2 : 1);
}

__global__ __launch_bounds__(kWG) void k_tile_count(const double *__restrict__ bbox, int ntiles, double sep_low,
                                                    int32_t *__restrict__ chunk_cnt) {
  __shared__ int part[kTileClasses][kWG];
  int c3[kTileClasses] = {0, 0, 0};
  const int t0 = blockIdx.x * kTileChunk + (int)threadIdx.x * kTilesPerThread;
  for (int k = 0; k < kTilesPerThread; ++k)
    if (t0 + k < ntiles) ++c3[tile_class(bbox, t0 + k, sep_low)];
  for (int c = 0; c < kTileClasses; ++c) part[c][threadIdx.x] = c3[c];
  __syncthreads();
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < kTileClasses; ++c) part[c][threadIdx.x] += part[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < kTileClasses) chunk_cnt[blockIdx.x * kTileClasses + threadIdx.x] = part[threadIdx.x][0];
}

__global__ __launch_bounds__(kWG) void k_tile_emit(const double *__restrict__ bbox, int ntiles, double sep_low,
                                                   const int32_t *__restrict__ chunk_cnt, int32_t *__restrict__ tile_cnt,
                                                   int32_t *__restrict__ tile_list) {
  __shared__ int pre[kTileClasses][kWG];
  __shared__ int off[kTileClasses];
  const int tid = (int)threadIdx.x;
  if (tid < kTileClasses) {
    int o = 0;
    for (int q = 0; q < (int)blockIdx.x; ++q) o += chunk_cnt[q * kTileClasses + tid];
    off[tid] = o;
  }
  int cls[kTilesPerThread];
  int c3[kTileClasses] = {0, 0, 0};
  const int t0 = blockIdx.x * kTileChunk + tid * kTilesPerThread;
  for (int k = 0; k < kTilesPerThread; ++k) {
    cls[k] = t0 + k < ntiles ? tile_class(bbox, t0 + k, sep_low) : -1;
    if (cls[k] >= 0) ++c3[cls[k]];
  }
  for (int c = 0; c < kTileClasses; ++c) pre[c][tid] = c3[c];
  __syncthreads();
  if (tid < kTileClasses) {  // exclusive scan over the threads, one class per thread
    int run = off[tid];
    for (int q = 0; q < kWG; ++q) {
      const int v = pre[tid][q];
      pre[tid][q] = run;
      run += v;
    }
    if ((int)blockIdx.x == (int)gridDim.x - 1) tile_cnt[tid] = run;
  }
  __syncthreads();
  int pos[kTileClasses] = {pre[0][tid], pre[1][tid], pre[2][tid]};
  for (int k = 0; k < kTilesPerThread; ++k) {
    const int c = cls[k];
    if (c >= 0) tile_list[(size_t)c * ntiles + pos[c]++] = t0 + k;
  }
}

// One workgroup of kPatWG threads per kPatRows rows (kPatRPW rows per wave;
// the rows lie in one block of 64 and take that block's box); lanes sweep
// the columns 64 at a time.  Row data are staged in LDS (broadcast reads).
// Few rows per wavefront keep many wavefronts in flight: each one's sweep is
// a chain of loads and ballots over the candidate blocks (L5 sphere, N =
// 20480: with 64 rows in 256 threads the preparation took 0.30 ms, with 32
// rows in 1024 threads 0.24 ms, and EMIT 38 us less).
// COUNT: rowcnt[i] = |pattern row i|, kindcnt[i][k] = pairs (i, j >= i) of
// class k.  EMIT: write (col, row, kind) at rowptr[i] in column order.
// Column blocks whose vertex box is farther from the row block's box than
// nf * (largest diameter in either block) can hold neither a touching pair
// (touching triangles share a point) nor a near pair (centroids lie in the
// boxes), so they are skipped without looking at their elements.
constexpr int kPatWG = 1024;                        // threads per workgroup of k_pattern
constexpr int kPatRows = 32;                        // rows per workgroup (divides 64)
constexpr int kPatRPW = kPatRows / (kPatWG / 64);   // rows per wavefront
static_assert(64 % kPatRows == 0 && kPatRPW >= 1, "pattern rows per workgroup");
template <bool EMIT>
__global__ __launch_bounds__(kPatWG) void k_pattern(const int4 *__restrict__ tri4, const double4 *__restrict__ cen4,
                                                 const double *__restrict__ bbox, int N, double nf2, int32_t *rowcnt,
                                                 int32_t *kindcnt, const int32_t *__restrict__ rowptr, int32_t *pcol,
                                                 int32_t *prow, int32_t *pkind) {
  __shared__ int4 s_tri[64];
  __shared__ double4 s_cen[64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int I0 = blockIdx.x * kPatRows;
  if (threadIdx.x < 64) {
    int i = min(I0 + (int)threadIdx.x, N - 1);
    s_tri[threadIdx.x] = tri4[i];
    s_cen[threadIdx.x] = cen4[i];
  }
  __syncthreads();
  int cnt[kPatRPW], base[kPatRPW];
  int kc[kPatRPW][4];
#pragma unroll
  for (int k = 0; k < kPatRPW; ++k) {
    cnt[k] = 0;
    kc[k][0] = kc[k][1] = kc[k][2] = kc[k][3] = 0;
    int i = I0 + w * kPatRPW + k;
    base[k] = (EMIT && i < N) ? rowptr[i] : 0;
  }
  const double *rb = bbox + 8 * (blockIdx.x / (64 / kPatRows));
  const int nblk = (N + 63) / 64;
  // Column blocks in rounds of kPatWG: the box tests of a round run in parallel
  // and the blocks that pass are listed in LDS in increasing order (wave
  // ballots, then the waves' counts in wave order), then swept.
  __shared__ int s_cand[kPatWG];
  __shared__ int s_wcnt[kPatWG / 64];
  for (int R0 = 0; R0 < nblk; R0 += kPatWG) {
    const int Jb = R0 + (int)threadIdx.x;
    bool keep = false;
    if (Jb < nblk) {
      const double *cb = bbox + 8 * Jb;
      const double thr = nf2 * fmax(rb[6], cb[6]);
      keep = !(box_dist2(rb, cb) > thr * (1.0 + 1e-9));
    }
    const uint64_t km = __ballot(keep);
    if (lane == 0) s_wcnt[w] = __popcll(km);
    __syncthreads();
    int off = 0, ncand = 0;
    for (int q = 0; q < kPatWG / 64; ++q) {
      if (q < w) off += s_wcnt[q];
      ncand += s_wcnt[q];
    }
    if (keep) s_cand[off + __popcll(km & ((1ull << lane) - 1ull))] = Jb;
    __syncthreads();
    ncand = __builtin_amdgcn_readfirstlane(ncand);
    for (int c = 0; c < ncand; ++c) {
      const int J0 = 64 * __builtin_amdgcn_readfirstlane(s_cand[c]);
      const int j = J0 + lane;
      const bool jv = j < N;
      int4 tj = tri4[jv ? j : N - 1];
      double4 cj = cen4[jv ? j : N - 1];
#pragma unroll
      for (int k = 0; k < kPatRPW; ++k) {
        const int i = I0 + w * kPatRPW + k;
        if (i < N) {  // uniform
          int cls = jv ? pair_class(s_tri[w * kPatRPW + k], s_cen[w * kPatRPW + k], tj, cj, nf2) : -1;
          uint64_t m = __ballot(cls >= 0);
          if (!EMIT) {
            cnt[k] += __popcll(m);
#pragma unroll
            for (int q = 0; q < 4; ++q) kc[k][q] += __popcll(__ballot(cls == q && j >= i));
          } else {
            if (cls >= 0) {
              int pos = base[k] + __popcll(m & ((1ull << lane) - 1ull));
              pcol[pos] = j;
              prow[pos] = i;
              pkind[pos] = cls;
            }
            base[k] += __popcll(m);
          }
        }
      }
    }
    __syncthreads();  // s_cand and s_wcnt are rewritten by the next round
  }
  if (!EMIT && lane == 0) {
#pragma unroll
    for (int k = 0; k < kPatRPW; ++k) {
      int i = I0 + w * kPatRPW + k;
      if (i < N) {
        rowcnt[i] = cnt[k];
        for (int q = 0; q < 4; ++q) kindcnt[4 * i + q] = kc[k][q];
      }
    }
  }
}

// Exclusive scan of the row counts (one workgroup of 1024 threads, each
// owning a contiguous chunk: chunk sums, an exclusive scan of them by wave
// scans and the waves' totals in wave order, then the chunk's row pointers)
// and the totals by class (integers: any summation order gives the same).
// info[0] = nnz, info[1..4] = coincident, edge, vertex, near pairs (i <= j);
// info[5] = 1 if nnz overflows int32.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ rowcnt,
                                               const int32_t *__restrict__ kindcnt, int N,
                                               int32_t *rowptr, int64_t *info) {
  __shared__ int64_t s_w[16];
  __shared__ int64_t s_wk[4][16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int chunk = (N + 1023) / 1024;
  const int b = min(N, t * chunk), e = min(N, b + chunk);
  int64_t s = 0, k[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int i = b; i < e; ++i) {
    s += rowcnt[i];
    const int4 kc = *reinterpret_cast<const int4 *>(kindcnt + 4 * i);
    k[0] += kc.x;
    k[1] += kc.y;
    k[2] += kc.z;
    k[3] += kc.w;
  }
  int64_t inc = s;  // inclusive scan over the wavefront's lanes
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t v = __shfl_up(inc, off, 64);
    if (lane >= off) inc += v;
  }
  for (int q = 0; q < 4; ++q)
    for (int off = 32; off >= 1; off >>= 1) k[q] += __shfl_xor(k[q], off, 64);
  if (lane == 63) s_w[w] = inc;
  if (lane == 0)
    for (int q = 0; q < 4; ++q) s_wk[q][w] = k[q];
  __syncthreads();
  int64_t woff = 0, tot = 0;
  for (int q = 0; q < 16; ++q) {
    if (q < w) woff += s_w[q];
    tot += s_w[q];
  }
  if (t == 0) {
    int64_t kt[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; ++q)
      for (int v = 0; v < 16; ++v) kt[q] += s_wk[q][v];
    info[0] = tot;
    info[1] = kt[3];
    info[2] = kt[2];
    info[3] = kt[1];
    info[4] = kt[0];
    info[5] = tot > 2147483647ll ? 1 : 0;
  }
  int64_t acc = woff + inc - s;
  for (int i = b; i < e; ++i) {
    rowptr[i] = (int32_t)acc;
    acc += rowcnt[i];
  }
  if (t == 1023) rowptr[N] = (int32_t)acc;
}

int launch_geometry(const double *verts, const int32_t *tris, int64_t N, int far_order,
                    void *mesh_ws, hipStream_t s) {
  FarRule r{};
  double x[8], w[8];
  gauss_legendre01(far_order, x, w);
  r.Q = far_order * far_order;
  for (int a = 0; a < far_order; ++a)
    for (int b = 0; b < far_order; ++b) {
      int k = a * far_order + b;
      r.s[k] = x[a];
      r.t[k] = x[b] * (1.0 - x[a]);
      r.w[k] = w[a] * w[b] * (1.0 - x[a]);
    }
  FarRule rL{};
  rL.Q = kQLow;
  radon7(rL.s, rL.t, rL.w);
  MeshLayout L(N);
  char *base = static_cast<char *>(mesh_ws);
  int grid = (int)((N + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_geometry, dim3(grid), dim3(kWG), 0, s, verts, tris, (int)N, r, rL,
                     reinterpret_cast<int4 *>(base + L.tri4), reinterpret_cast<double4 *>(base + L.cen4),
                     reinterpret_cast<double *>(base + L.area), reinterpret_cast<double4 *>(base + L.qpA64),
                     reinterpret_cast<double *>(base + L.qpS64), reinterpret_cast<float4 *>(base + L.qpA32),
                     reinterpret_cast<float *>(base + L.qpS32), reinterpret_cast<double4 *>(base + L.qpLA64),
                     reinterpret_cast<double *>(base + L.qpLS64));
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

int launch_pattern(const double *verts, const int32_t *tris, int64_t N, double near_factor, const void *mesh_ws,
                   void *pattern, int64_t nnz, int32_t precision, bool emit, hipStream_t s) {
  (void)tris;
  MeshLayout L(N);
  char *base = static_cast<char *>(const_cast<void *>(mesh_ws));
  const int4 *tri4 = reinterpret_cast<const int4 *>(base + L.tri4);
  const double4 *cen4 = reinterpret_cast<const double4 *>(base + L.cen4);
  int32_t *rowcnt = reinterpret_cast<int32_t *>(base + L.rowcnt);
  int32_t *kindcnt = reinterpret_cast<int32_t *>(base + L.kindcnt);
  int32_t *rowptr = reinterpret_cast<int32_t *>(base + L.rowptr);
  double nf2 = near_factor * near_factor;
  int grid = (int)((N + 63) / 64);
  const double *bbox = reinterpret_cast<const double *>(base + L.blockbox);
  const unsigned pgrid = (unsigned)((N + kPatRows - 1) / kPatRows);
  if (!emit) {
    hipLaunchKernelGGL(k_blockbox, dim3(grid), dim3(64), 0, s, verts, tri4, cen4, (int)N, const_cast<double *>(bbox));
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
    const int64_t ntiles = far_tiles(N);
    const unsigned nchunk = (unsigned)((ntiles + kTileChunk - 1) / kTileChunk);
    int32_t *tile_cnt = reinterpret_cast<int32_t *>(base + L.tiles);
    int32_t *tile_list = tile_cnt + 16;
    int32_t *chunk_cnt = tile_list + kTileClasses * ntiles;
    hipLaunchKernelGGL(k_colpoints, dim3((unsigned)((N + kWG - 1) / kWG)), dim3(kWG), 0, s,
                       reinterpret_cast<const double *>(base + L.qpS64), reinterpret_cast<const double *>(base + L.qpLS64),
                       bbox, (int)N, reinterpret_cast<float *>(base + L.qpB16), reinterpret_cast<float *>(base + L.qpBL));
    const double sep_low = precision == BC_FP64 ? kSepFarLow64 : kSepFarLow;
    hipLaunchKernelGGL(k_tile_count, dim3(nchunk), dim3(kWG), 0, s, bbox, (int)ntiles, sep_low, chunk_cnt);
    hipLaunchKernelGGL(k_tile_emit, dim3(nchunk), dim3(kWG), 0, s, bbox, (int)ntiles, sep_low,
                       (const int32_t *)chunk_cnt, tile_cnt, tile_list);
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
    hipLaunchKernelGGL(k_pattern<false>, dim3(pgrid), dim3(kPatWG), 0, s, tri4, cen4, bbox, (int)N, nf2, rowcnt, kindcnt,
                       (const int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr);
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, rowcnt, kindcnt, (int)N, rowptr,
                       reinterpret_cast<int64_t *>(base + L.info));
  } else {
    PatternLayout P(N, nnz, precision);
    char *pb = static_cast<char *>(pattern);
    if (hipMemcpyAsync(pb + P.rowptr, rowptr, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return BC_EDEVICE;
    hipLaunchKernelGGL(k_pattern<true>, dim3(pgrid), dim3(kPatWG), 0, s, tri4, cen4, bbox, (int)N, nf2, (int32_t *)nullptr,
                       (int32_t *)nullptr, (const int32_t *)rowptr, reinterpret_cast<int32_t *>(pb + P.col),
                       reinterpret_cast<int32_t *>(pb + P.row), reinterpret_cast<int32_t *>(pb + P.kind));
  }
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
