// Internal layouts shared by the host library and the gfx950 kernels.
//
// A model lives in device memory as a handful of pools:
//   ctrl   : stored control points of all blocks, C order [n0][n1][n2] per
//            block, blocks back to back (storage type FP32 / BF16 / FP16);
//   rec    : one SpanRec per (block, axis, span), the FP64 data of the span
//            rule and of the local coordinate plus the FP32 chain-rule scale;
//   mats   : deduplicated FP32 tables of the polynomial pieces of the basis
//            functions on a span (value and d/dtau coefficients);
//   blocks : one DevBlock per block;
//   edges  : FP64 block edges per axis.
// Everything the kernels need about a single-block model (the common case)
// is also copied into the kernel argument (DevModel::b0) so it is uniform.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace mfa {

constexpr int kMaxDegree = 7;

// One knot span [t, t_next) of one axis of one block (span index s = p + j).
struct SpanRec {
  double t;        // T[s]
  double t_next;   // T[s+1]
  double inv_h;    // 1 / (T[s+1] - T[s])  (FP64 division on the host)
  float dscale;    // (float)(inv_h * inv_ext): d/dtau -> d/dworld
  int32_t mat;     // index of the basis table in the matrix pool
};
static_assert(sizeof(SpanRec) == 32, "SpanRec layout");

struct DevBlock {
  double lo[3];         // world box of the block
  double inv_ext[3];    // 1 / (hi - lo), FP64 division on the host
  int64_t ctrl_off;     // element offset of the block's control points
  int32_t n[3];         // control points per axis
  int32_t nsp[3];       // spans per axis = n - p
  int32_t rec_off[3];   // index of the block's span 0 record per axis
  int32_t rs1;          // row stride along axis 1 in elements (n2, padded to
                        // even for 16-bit storage so rows pair into dwords)
  int32_t mc[3];        // macro cells per axis = ceil(nsp / 2^mc_shift)
  int32_t mc_off;       // index of the block's first macro cell in the bounds pool
  double ext[3];        // hi - lo (estimates of cell exits only)
  int32_t tile_off;     // first sort bucket of the block
  int32_t sc_off[2];    // per super-cell level: the block's first cell in that level's pool
  int32_t sc[2][3];     // per level: cells per axis = ceil(nsp / 2^sc_shift[level])
  int32_t pad;
};
static_assert(sizeof(DevBlock) == 176, "DevBlock layout");

// Points sorted for decode are grouped by (block, tile); a tile spans
// 2^sort_shift knot spans per axis, the shift chosen per model: the largest
// whose control-point windows fit kWinMax values, made larger while the
// model would have more than kMaxBuckets buckets.
constexpr int kMaxBuckets = 32768;
static_assert(kMaxBuckets <= 65536, "bucket ids are carried in 16 bits");

// Sorted decode works on items of at most kTilePoints consecutive sorted
// points of one bucket (a bucket of c points is cut into ceil(c /
// kTilePoints) items of equal size).  The control points the exact spans of
// a bucket's points can touch (the tile's spans plus p per axis) form a
// window that is staged in LDS when it holds at most kWinMax values; a point
// whose exact spans leave the window (a span guess that rounding moved into
// the neighbouring tile, or non-uniform knots) reads its rows from global
// memory.
constexpr int kTilePoints = 4096;

// Up to kOneLevelBuckets buckets the points are scattered to their buckets
// in one pass; above, in two: first by coarse key bucket >> fine_shift (at
// most kCoarseBuckets keys, runs of hundreds of records per chunk), then
// within the coarse runs by bucket.
constexpr int kOneLevelBuckets = 1024;
constexpr int kCoarseBuckets = 64;
// The coarse cursors sit one per 128-byte line: every chunk updates all of
// them, and 64 counters in two lines would put every atomic of the pass on
// the same two L2 channels.
constexpr int kCursorStride = 32;
constexpr int kWinMax = 8192;

// Size of the file-scope device scratch of the allocation-free sorted
// decode (one copy per device, held until the process ends).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;

// Per-block data of the bucket computation of multi-block models, staged in
// LDS by the sort kernels (models of at most kSortBlkLds blocks and
// kSortEdgesLds block edges).  The bucket only orders the work, so it is
// computed in FP32 (lo and nsp / (hi - lo) rounded to FP32); the decode
// checks each point's exact FP64 owner against the bucket's block.
struct SortBlk {
  float lo[3];
  float tscale[3];       // (nsp / (hi - lo)) / 2^sort_shift: tiles per unit length
  int32_t nt[3];         // tiles per axis, ceil(nsp / 2^sort_shift)
  int32_t tile_off;
  int32_t pad[2];
};
static_assert(sizeof(SortBlk) == 48, "SortBlk layout");
constexpr int kSortBlkLds = 512;
constexpr int kSortEdgesLds = 256;

struct BucketWin {
  int32_t block;        // owning block
  int32_t o[3];         // first control index of the window per axis
  int32_t w[3];         // window extent per axis (control points)
  int32_t pad;
};
static_assert(sizeof(BucketWin) == 32, "BucketWin layout");

// Spans per axis grouped into one macro cell for the value bounds used to
// skip samples that the transfer function makes fully transparent: 2^shift,
// shift in [0, kMaxMacroShift], chosen per model (DevModel::mc_shift).
constexpr int kMaxMacroShift = 2;

// Two coarser levels of the same bounds, super cells of 2^3 and 2^2 macro
// cells per axis, let a ray cross the transparent stretch in front of its
// first visible cell in a few leaps.
constexpr int kSuperShift[2] = {3, 2};

// Kernel family of a model: single block with uniform knots, single block
// with a non-uniform axis (span guess tables), several blocks.
constexpr int kKindPlain = 0, kKindGraded = 1, kKindMulti = 2;

struct DevModel {
  const void* ctrl;
  const SpanRec* rec;
  const float* mats;
  const DevBlock* blocks;
  const double* edges;   // axis 0 (grid0+1 values), then axis 1, then axis 2
  int64_t ctrl_bytes;    // size of the ctrl pool (buffer range)
  int32_t edge_off[3];
  int32_t grid[3];
  int32_t nblocks;
  int32_t mat_stride;    // floats per basis table
  int32_t n_mats;        // basis tables in the pool
  int32_t n_rec;         // span records in the pool
  int32_t imat;          // id of the uniform interior table (UniformTable), or -1
  int32_t mc_shift;      // log2 of the spans per macro cell and axis
  int32_t sort_shift;    // log2 of the spans per sort tile and axis
  const BucketWin* bwin;  // per sort bucket: control-point window
  int32_t win_max;       // largest window (values)
  const SortBlk* sblk;   // per block: data of the sort-bucket computation
  const float* sedges;   // the block edges rounded to FP32 (sort only)
  int32_t n_edges;       // block edges over the three axes
  const uint32_t* mcb;   // per macro cell (lo, hi) bounds of the stored values as
                         // two FP16 halves rounded outward, widened by a margin
                         // covering FP32 evaluation error
  const uint32_t* scb[2];  // the same bounds per super cell, coarse level first
  // span guess tables of the non-uniform knot axes (nullptr: none): for
  // block b and axis a, gmeta[6 b + a] = offset of the axis's table in gtab
  // (-1: uniform knots, guess floor(u * nsp)) and gmeta[6 b + 3 + a] = its
  // bin count G; gtab[offset + floor(u * G)] is the span (record index)
  // holding u = g / G, the bins being narrower than the shortest span
  const int32_t* gtab;
  const int32_t* gmeta;
  int32_t sc_shift[2];     // log2 of the spans per super cell and axis, per level
  double edge_scale[3];  // grid[a] / (E[G] - E[0]): block-owner guess only
  double box_lo[3];
  double box_hi[3];
  DevBlock b0;           // block 0 (the only block of single-block models)
};

// Storage element types.
enum class Storage : int { F32 = 1, BF16 = 2, F16 = 3 };

// Basis table of degree p for one span: value coefficients c[r][m]
// (function r = 0..p, power m = 0..p, ascending) followed by derivative
// coefficients e[r][m] = (m+1) c[r][m+1] (m = 0..p-1); padded to 4 floats.
inline constexpr int mat_stride(int p) {
  return (((p + 1) * (p + 1) + (p + 1) * p) + 3) / 4 * 4;
}

// The basis table of an interior span of uniform knots (the uniform
// B-spline pieces of degree p), computed at compile time by the Cox-de Boor
// recursion on polynomials in tau over the integer knots -p..p+1, in FP64,
// then rounded to FP32.  Host and kernels use this one routine, so a span
// whose table equals it can be evaluated from literals.
template <int P>
struct UniformTable {
  float c[mat_stride(P)];
  constexpr UniformTable() : c() {
    double N[P + 1][P + 1] = {};   // N[r][m]: function r, power m of tau
    double M[P + 1][P + 1] = {};
    N[0][0] = 1.0;
    for (int q = 1; q <= P; ++q) {
      for (int r = 0; r <= P; ++r)
        for (int m = 0; m <= P; ++m) M[r][m] = 0.0;
      for (int r = 0; r <= q; ++r) {
        // knots t_i = i relative to the span start; function i = r - q
        const int i = r - q;
        if (r >= 1) {            // (u - t_i) / q * N_{i,q-1}, u = tau
          const double a0 = (0.0 - i) / q, a1 = 1.0 / q;
          for (int m = 0; m <= P; ++m) {
            M[r][m] += a0 * N[r - 1][m];
            if (m + 1 <= P) M[r][m + 1] += a1 * N[r - 1][m];
          }
        }
        if (r <= q - 1) {        // (t_{i+q+1} - u) / q * N_{i+1,q-1}
          const double b0 = (double)(i + q + 1) / q, b1 = -1.0 / q;
          for (int m = 0; m <= P; ++m) {
            M[r][m] += b0 * N[r][m];
            if (m + 1 <= P) M[r][m + 1] += b1 * N[r][m];
          }
        }
      }
      for (int r = 0; r <= P; ++r)
        for (int m = 0; m <= P; ++m) N[r][m] = M[r][m];
    }
    for (int r = 0; r <= P; ++r)
      for (int m = 0; m <= P; ++m) c[r * (P + 1) + m] = (float)N[r][m];
    for (int r = 0; r <= P; ++r)
      for (int m = 0; m < P; ++m) c[(P + 1) * (P + 1) + r * P + m] = (float)((m + 1) * N[r][m + 1]);
  }
};

struct SortArgs {
  const float* xyz;      // input SoA [3][n]
  int64_t n;
  float4* rec;           // [n] sorted records (x, y, z, input index as bits)
  uint32_t* hist;        // [nb] points per bucket
  uint32_t* start;       // [nb + 1] first sorted position of each bucket; start[nb] = n
  uint32_t* cursor;      // [nb] positions handed out so far per bucket
  int2* items;           // [<= n / kTilePoints + nb] (bucket, part) per decode item
  int32_t* n_items;      // number of items
  int32_t nb;            // buckets (<= kMaxBuckets)
  // two-level split (nb > kOneLevelBuckets): records grouped by coarse key
  // (bucket >> fine_shift) first, then by bucket
  int32_t fine_shift;
  float4* tmp;           // [n] records in coarse order, or null (one level)
  uint32_t* ccursor;     // [kCoarseBuckets * kCursorStride] positions handed out per coarse key
  // two-level split, results through the coarse order (or null): the
  // coarse pass writes each point's position in tmp here (in input order),
  // the bucket pass gives each record that position instead of the input
  // index, the decode writes its results at it (into tmp, no longer read),
  // and a last pass gathers them back into input order
  uint32_t* tpos;        // [n]
  // with tpos: the histogram pass writes each point's bucket here (in input
  // order, in the region of rec, which the bucket pass fills only later);
  // the coarse pass carries it in the record's fourth word to the bucket
  // pass, so that neither recomputes it
  uint16_t* bkt;         // [n]
};

struct GridArgs {
  const double* axis[3];
  int32_t res[3];
  int32_t ta;            // grid entries along axis 0 per wave
  float* out;
  int32_t* spans;
};

struct RenderArgs {
  const float* tf;
  float* rgba;
  int32_t* nsamp;
  int32_t* neval;
  float* alpha;
  int32_t alpha_stride;
  int32_t w, h;
  int32_t kind;
  int32_t max_samples;
  int32_t shininess;
  float vmin, inv_range;   // TF domain: s = (f - vmin) * inv_range * 255
  float ert_alpha;
  float ka, kd, ks, g0;
  double eye[3], fwd[3], right[3], up[3];
  double sx, sy, step;
  double inv_step;        // 1 / step (estimates only)
  // partial render (object-space split): composite only the samples owned
  // by blocks in [reg_lo, reg_hi) per axis, whose world box is
  // [reg_box_lo, reg_box_hi]; key[pixel] = entry parameter of the ray into
  // that box (+inf when the ray misses it or the model box)
  int32_t partial;
  int32_t reg_lo[3], reg_hi[3];
  double reg_box_lo[3], reg_box_hi[3];
  double* key;
  // isosurface render: level and surface colour; key[pixel] = hit
  // parameter t* (+inf without a hit), nsamp = (K, hit sample or -1)
  float iso;
  float iso_rgb[3];
};

// Volume of samples on a uniform grid rendered through a local filter:
// sample (i0, i1, i2) at lo + i * h, h = (hi - lo) / (n - 1) (FP64 on the
// host); v = nullptr for the analytic Marschner-Lobb field.
struct VolArgs {
  const float* v;
  int32_t n[3];
  double lo[3], hi[3], h[3];
  double inv_hd[3];      // 1 / h (FP64 division on the host)
  float inv_h[3];
  int64_t bytes;         // sample bytes; stencil rows by buffer loads below 4 GiB
};

// Depth-ordered compositing of up to kMaxPartials partial images.
constexpr int kMaxPartials = 16;

struct CompositeArgs {
  const float4* images[kMaxPartials];   // [npix] premultiplied RGBA each
  const double* keys[kMaxPartials];     // [npix] depth key each (+inf: empty)
  int32_t g;
  int64_t npix;
  float4* out;
};

}  // namespace mfa

namespace mfa {

// Serving: a batch is a list of equal work items over admitted requests.
// A render item is one 16x16 pixel tile of a frame; a points item is 256
// consecutive points of a query set.
enum { kServeRender = 0, kServePoints = 1 };

struct ServeReq {
  int32_t kind;          // kServeRender / kServePoints
  int32_t model;         // index in the device model table
  RenderArgs ra;         // render requests
  const float* xyz;      // points requests: device SoA [3][n]
  float* out;            //                  device [n][4]
  int64_t n;
};

struct ServeItem {
  int32_t req;           // index in the batch's request array
  int32_t index;         // tile or 256-point chunk of the request
};

}  // namespace mfa
