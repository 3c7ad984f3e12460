// gfx950 kernels of the MFA evaluator and ray caster.
//
// Per sample (paper Sec. III-A model, Sec. IV-A4 query + ray casting):
//   world x (FP64) -> owning block -> parameter u (FP64) -> knot span (FP64
//   compares against the stored knots) -> local coordinate tau (FP64, then
//   FP32) -> basis values and d/dtau from the span's polynomial table (FP32)
//   -> sum-factorised (p+1)^3 contraction for value and three partials
//   (FP32 accumulate; control points FP32 / BF16 / FP16) -> chain rule.
// The renderer adds transfer function, headlight Phong, front-to-back "over"
// (Sec. IV-A5) and early termination tested once per step on the wave.
//
// Exact FP64 steps are written with contraction off so they round exactly
// like the reference definitions (one rounding per operation).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "mfa.h"
#include "mfa_internal.h"

namespace mfa {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kBlock = 256;

// ------------------------------------------------------------------ memory
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int64_t bytes) {
  const int64_t cap = 0xFFFFFFFFll;
  const uint32_t nrec = (uint32_t)(bytes < cap ? bytes : cap);
  // word 3 = 0x00020000: raw (untyped) buffer on gfx9-class targets
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nrec, 0x00020000);
}

// Loads N consecutive 32-bit words at byte offset vo (per lane) + so (uniform).
template <int N>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so,
                                           uint32_t* w) {
  if constexpr (N >= 4) {
    u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0);
    w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
    load_words<N - 4>(rs, vo + 16, so, w + 4);
  } else if constexpr (N == 3) {
    u32x3 q = __builtin_amdgcn_raw_buffer_load_b96(rs, vo, so, 0);
    w[0] = q.x; w[1] = q.y; w[2] = q.z;
  } else if constexpr (N == 2) {
    u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0);
    w[0] = q.x; w[1] = q.y;
  } else if constexpr (N == 1) {
    w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0);
  }
}

// One row of P+1 control points along axis 2 starting at element e (per
// lane) + es (uniform): load() fetches the raw words, unpack() converts them
// to FP32, so a caller can put every load of a sample in flight before the
// first conversion waits for one.
template <int P, Storage S>
struct Row;

template <int P>
struct Row<P, Storage::F32> {
  static constexpr int kElem = 4;
  static constexpr int kWords = P + 1;
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t e, uint32_t es,
                                              uint32_t (&w)[kWords]) {
    load_words<P + 1>(rs, e * 4u, es * 4u, w);
  }
  static __device__ __forceinline__ void unpack(const uint32_t (&w)[kWords], uint32_t,
                                                float (&v)[P + 1]) {
#pragma unroll
    for (int k = 0; k <= P; ++k) v[k] = __uint_as_float(w[k]);
  }
};

// 16-bit rows: the dword-aligned window holding elements e..e+P, funnel-
// shifted by one half-word when e is odd (e and the uniform part of the
// offset are even-aligned together: row strides are even).
template <int P>
struct Halves {
  static constexpr int kOut = (P + 2) / 2;   // dwords holding P+1 halves
  static constexpr int kWords = kOut + 1;
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t e, uint32_t es,
                                              uint32_t (&w)[kWords]) {
    load_words<kWords>(rs, (e & ~1u) * 2u, es * 2u, w);
  }
  static __device__ __forceinline__ void align(const uint32_t (&w)[kWords], uint32_t e,
                                               uint32_t (&h)[kOut]) {
    const uint32_t sh = (e & 1u) * 16u;
#pragma unroll
    for (int q = 0; q < kOut; ++q) h[q] = __builtin_amdgcn_alignbit(w[q + 1], w[q], sh);
  }
};

template <int P>
struct Row<P, Storage::BF16> : Halves<P> {
  static constexpr int kElem = 2;
  static __device__ __forceinline__ void unpack(const uint32_t (&w)[Halves<P>::kWords], uint32_t e,
                                                float (&v)[P + 1]) {
    uint32_t h[Halves<P>::kOut];
    Halves<P>::align(w, e, h);
#pragma unroll
    for (int k = 0; k <= P; ++k)
      v[k] = (k & 1) ? __uint_as_float(h[k >> 1] & 0xFFFF0000u) : __uint_as_float(h[k >> 1] << 16);
  }
};

template <int P>
struct Row<P, Storage::F16> : Halves<P> {
  static constexpr int kElem = 2;
  static __device__ __forceinline__ void unpack(const uint32_t (&w)[Halves<P>::kWords], uint32_t e,
                                                float (&v)[P + 1]) {
    uint32_t h[Halves<P>::kOut];
    Halves<P>::align(w, e, h);
#pragma unroll
    for (int k = 0; k <= P; ++k) {
      const unsigned short bits = (k & 1) ? (unsigned short)(h[k >> 1] >> 16)
                                          : (unsigned short)(h[k >> 1] & 0xFFFFu);
      v[k] = __half2float(__ushort_as_half(bits));
    }
  }
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Streaming 16-byte store: the line bypasses the caches.  Only for outputs
// written in whole lines (scattered 16-byte writes become twice as slow).
__device__ __forceinline__ void store_stream(float4* p, float4 v) {
  const f32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
}

// ------------------------------------------------------------------ FP64 decisions
__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return fmin(fmax(v, lo), hi);
}

// Span rule s = max{ i in [p, n-1] : T[i] <= u } over the span records
// R[0..nsp-1] of one axis (record j describes span s = p + j), in steps so
// that the record loads of the three axes of a point can be in flight
// together: guess_span() takes floor(u * nsp), span_ok() checks the guess by
// exact comparisons with the stored knots, and fix_span() walks to the exact
// span where the check fails (u within rounding of a knot, or non-uniform
// knots).
__device__ __forceinline__ int guess_span(int nsp, double u) {
  const int j = (int)(u * (double)nsp);
  return j < 0 ? 0 : (j > nsp - 1 ? nsp - 1 : j);
}

// The guess of a point's span on axis a of block B: floor(u * nsp) for
// uniform knots, else the span of u's bin in the axis's guess table (the
// exact span or the one before it).  GT: the single-block kernels built for
// models with a non-uniform axis; every other kernel compiles the plain
// guess alone (the table path, even untaken, costs the multi-block kernels
// about 10 %), and a non-uniform axis there is found by the walk.
template <bool GT>
__device__ __forceinline__ int guess_span(const DevModel& m, const DevBlock* __restrict__ B,
                                          int block, int a, double u) {
  if constexpr (!GT) return guess_span(B->nsp[a], u);
  if (m.gtab == nullptr) return guess_span(B->nsp[a], u);   // no table in the model (scalar test)
  const int off = m.gmeta[6 * block + a];
  if (off < 0) return guess_span(B->nsp[a], u);
  const int G = m.gmeta[6 * block + 3 + a];
  const int g = (int)(u * (double)G);
  return m.gtab[off + (g < 0 ? 0 : (g > G - 1 ? G - 1 : g))];
}

__device__ __forceinline__ bool span_ok(int nsp, double u, int j, const SpanRec& rec) {
  return !(j < nsp - 1 && rec.t_next <= u) & !(j > 0 && rec.t > u);
}

__device__ __forceinline__ void fix_span(const SpanRec* __restrict__ R, int nsp, double u, int& j,
                                         SpanRec& rec) {
  while (j < nsp - 1 && rec.t_next <= u) { ++j; rec = R[j]; }
  while (j > 0 && rec.t > u) { --j; rec = R[j]; }
}

__device__ __forceinline__ int locate_span(const SpanRec* __restrict__ R, int nsp, double u,
                                           SpanRec& rec) {
  int j = guess_span(nsp, u);
  rec = R[j];
  if (!span_ok(nsp, u, j, rec)) fix_span(R, nsp, u, j, rec);
  return j;
}

// Local coordinate of u in its span, FP64 then rounded once to FP32.
__device__ __forceinline__ float local_tau(const SpanRec& rec, double u) {
#pragma clang fp contract(off)
  return (float)((u - rec.t) * rec.inv_h);
}

// Parameter of a world coordinate in its block (clamped box coordinate).
__device__ __forceinline__ double param_of(double xc, double lo, double inv_ext) {
#pragma clang fp contract(off)
  return clampd((xc - lo) * inv_ext, 0.0, 1.0);
}

// ------------------------------------------------------------------ basis
// Values N[r] and d/dtau D[r] (r = 0..P) of the basis functions active on a
// span, by Horner on the span's polynomial table (see mat_stride()).
template <int P>
using Table = float[mat_stride(P)];

template <int P>
__device__ __forceinline__ void load_table(const float* __restrict__ M, Table<P>& c) {
#pragma unroll
  for (int q = 0; q < mat_stride(P) / 4; ++q) {
    const float4 v = reinterpret_cast<const float4*>(M)[q];
    c[4 * q + 0] = v.x;
    c[4 * q + 1] = v.y;
    c[4 * q + 2] = v.z;
    c[4 * q + 3] = v.w;
  }
}

template <int P>
__device__ __forceinline__ void horner(const Table<P>& c, float tau, float (&N)[P + 1],
                                       float (&D)[P + 1]) {
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    float v = c[r * (P + 1) + P];
#pragma unroll
    for (int m = P - 1; m >= 0; --m) v = fmaf(v, tau, c[r * (P + 1) + m]);
    N[r] = v;
    const int e = (P + 1) * (P + 1) + r * P;
    float d = c[e + P - 1];
#pragma unroll
    for (int m = P - 2; m >= 0; --m) d = fmaf(d, tau, c[e + m]);
    D[r] = d;
  }
}

// Spans with the uniform interior table (imat) use it as literals; per-lane
// tables are loaded only when a lane of the wave sits on another span type.
template <int P>
__device__ __forceinline__ void basis(const float* __restrict__ mats, int stride, int mat, int imat,
                                      float tau, float (&N)[P + 1], float (&D)[P + 1]) {
  if (__all(mat == imat)) {
    constexpr UniformTable<P> U{};
    horner<P>(U.c, tau, N, D);
  } else {
    Table<P> c;
    load_table<P>(mats + mat * stride, c);
    horner<P>(c, tau, N, D);
  }
}

// ------------------------------------------------------------------ contraction
// f = sum_ijk Nx_i Ny_j Nz_k P_ijk and the three partials with one factor
// replaced by its derivative, summed axis 2 first, then axis 1, then axis 0.
// row(i, j, v) fills v with the P+1 control points P[i0+i][j0+j][k0..k0+P];
// every source of rows goes through this one summation order, so results do
// not depend on where the rows come from.
template <int P, class RowFn>
__device__ __forceinline__ void contract_rows(RowFn row, const float (&Nx)[P + 1],
                                              const float (&Dx)[P + 1], const float (&Ny)[P + 1],
                                              const float (&Dy)[P + 1], const float (&Nz)[P + 1],
                                              const float (&Dz)[P + 1], float& f, float& fx,
                                              float& fy, float& fz) {
  f = fx = fy = fz = 0.f;
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    float y = 0.f, yy = 0.f, yz = 0.f;
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      float v[P + 1];
      row(i, j, v);
      float z = 0.f, zd = 0.f;
#pragma unroll
      for (int k = 0; k <= P; ++k) {
        z = fmaf(Nz[k], v[k], z);
        zd = fmaf(Dz[k], v[k], zd);
      }
      y = fmaf(Ny[j], z, y);
      yy = fmaf(Dy[j], z, yy);
      yz = fmaf(Ny[j], zd, yz);
    }
    f = fmaf(Nx[i], y, f);
    fx = fmaf(Dx[i], y, fx);
    fy = fmaf(Nx[i], yy, fy);
    fz = fmaf(Nx[i], yz, fz);
  }
}

// The (P+1)^2 control rows of a located point from the control-point pool
// in global memory, kept as raw words so that all loads of a sample are in
// flight before the first use.  e0: element index of P[i0][j0][k0] (per
// lane); rows at + i*s0 + j*s1 (even for 16-bit storage, so every row has
// the parity of e0).  UNIFORM_STRIDES: s0, s1 are wave-uniform and go into
// the scalar offset.
template <int P, Storage S, bool UNIFORM_STRIDES>
struct Rows {
  uint32_t w[P + 1][P + 1][Row<P, S>::kWords];
  uint32_t e0;
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t e, uint32_t s0,
                                       uint32_t s1) {
    e0 = e;
#pragma unroll
    for (int i = 0; i <= P; ++i)
#pragma unroll
      for (int j = 0; j <= P; ++j) {
        if constexpr (UNIFORM_STRIDES)
          Row<P, S>::load(rs, e, (uint32_t)i * s0 + (uint32_t)j * s1, w[i][j]);
        else
          Row<P, S>::load(rs, e + (uint32_t)i * s0 + (uint32_t)j * s1, 0u, w[i][j]);
      }
  }
  __device__ __forceinline__ void get(int i, int j, float (&v)[P + 1]) const {
    Row<P, S>::unpack(w[i][j], e0, v);
  }
};

// ------------------------------------------------------------------ point location
// Owning block along one axis: b = max{ i in [0, G-1] : E[i] <= xc }, in
// the same steps as the span rule (guess from the mean block width, one
// exact check against the two bracketing edges, a walk only where it fails),
// so the edge loads of the three axes are in flight together.
__device__ __forceinline__ int guess_owner(const double* __restrict__ E, int G, double scale,
                                           double xc) {
  const int b = (int)((xc - E[0]) * scale);
  return b < 0 ? 0 : (b > G - 1 ? G - 1 : b);
}

__device__ __forceinline__ bool owner_ok(int G, double xc, int b, double e0, double e1) {
  return !(b < G - 1 && e1 <= xc) & !(b > 0 && e0 > xc);
}

__device__ __forceinline__ void fix_owner(const double* __restrict__ E, int G, double xc, int& b) {
  while (b < G - 1 && E[b + 1] <= xc) ++b;
  while (b > 0 && E[b] > xc) --b;
}

// Everything the evaluation needs about one world point after the exact
// FP64 steps: per axis the span, local coordinate, chain-rule scale and
// basis table; the first control row and the row strides; the macro cell.
struct Loc {
  float tau[3], ds[3];
  int mat[3], j[3];
  int block;
  uint32_t e0, s0, s1;
  int mc;
};

// A point after the exact FP64 map: owning block, parameters, and per axis
// the guessed span with its record (loads issued, not yet waited for).
struct Probe {
  const DevBlock* B;
  double u[3];
  SpanRec rec[3];
  int j[3];
  int b[3];        // owning block per axis (0 for single-block models)
  int block;
};

// Macro cell of the spans j of block B.
__device__ __forceinline__ int macro_cell(const DevModel& m, const DevBlock* __restrict__ B,
                                          const int (&j)[3]) {
  const int sh = m.mc_shift;
  return B->mc_off + (((j[0] >> sh) * B->mc[1] + (j[1] >> sh)) * B->mc[2] + (j[2] >> sh));
}

// Owning block of a point of a multi-block model (EDG: the block edges,
// m.edges or an LDS copy): q.block and q.b, and the clamped coordinates.
__device__ __forceinline__ void probe_owner(const DevModel& m, const double (&x)[3],
                                            const double* __restrict__ EDG, Probe& q,
                                            double (&xc)[3]) {
  int b[3];
  double e0[3], e1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* E = EDG + m.edge_off[a];
    xc[a] = clampd(x[a], E[0], E[m.grid[a]]);
    b[a] = guess_owner(E, m.grid[a], m.edge_scale[a], xc[a]);
    e0[a] = E[b[a]];
    e1[a] = E[b[a] + 1];
  }
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) ok &= owner_ok(m.grid[a], xc[a], b[a], e0[a], e1[a]);
  if (!ok) {
#pragma unroll
    for (int a = 0; a < 3; ++a) fix_owner(EDG + m.edge_off[a], m.grid[a], xc[a], b[a]);
  }
  q.block = (b[0] * m.grid[1] + b[1]) * m.grid[2] + b[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) q.b[a] = b[a];
}

// The rest of the probe once the point's block record B is known: the
// parameters and the guessed spans with their records (loads issued).
template <bool GT = false>
__device__ __forceinline__ void probe_spans(const DevModel& m, const SpanRec* __restrict__ R,
                                            const double (&xc)[3], const DevBlock* B, Probe& q) {
  q.B = B;
#pragma unroll
  for (int a = 0; a < 3; ++a) q.u[a] = param_of(xc[a], B->lo[a], B->inv_ext[a]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.j[a] = guess_span<GT>(m, B, q.block, a, q.u[a]);
    q.rec[a] = R[B->rec_off[a] + q.j[a]];
  }
}

// R: span records (global pool or its LDS copy); EDG: the block edges
// (m.edges or an LDS copy).
template <bool MULTI, bool GT = false>
__device__ __forceinline__ Probe probe(const DevModel& m, const SpanRec* __restrict__ R,
                                       const double (&x)[3], const double* __restrict__ EDG) {
  Probe q;
  q.B = &m.b0;
  if constexpr (MULTI) {
    double xc[3];
    probe_owner(m, x, EDG, q, xc);
    probe_spans<GT>(m, R, xc, m.blocks + q.block, q);
    return q;
  } else {
    q.block = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q.b[a] = 0;
      q.u[a] = param_of(clampd(x[a], m.box_lo[a], m.box_hi[a]), m.box_lo[a], q.B->inv_ext[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.j[a] = guess_span<GT>(m, q.B, q.block, a, q.u[a]);
    q.rec[a] = R[q.B->rec_off[a] + q.j[a]];
  }
  return q;
}

template <bool MULTI, bool GT = false>
__device__ __forceinline__ Probe probe(const DevModel& m, const SpanRec* __restrict__ R,
                                       const double (&x)[3]) {
  return probe<MULTI, GT>(m, R, x, m.edges);
}

// Exact spans (a walk only where a guess fails its check), local
// coordinates, first control row and macro cell of a probed point.
__device__ __forceinline__ Loc finish(const DevModel& m, const SpanRec* __restrict__ R, Probe& q) {
  const DevBlock* __restrict__ B = q.B;
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) ok &= span_ok(B->nsp[a], q.u[a], q.j[a], q.rec[a]);
  if (!ok) {
#pragma unroll
    for (int a = 0; a < 3; ++a) fix_span(R + B->rec_off[a], B->nsp[a], q.u[a], q.j[a], q.rec[a]);
  }
  Loc L;
  L.block = q.block;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    L.j[a] = q.j[a];
    L.tau[a] = local_tau(q.rec[a], q.u[a]);
    L.ds[a] = q.rec[a].dscale;
    L.mat[a] = q.rec[a].mat;
  }
  const uint32_t n1 = (uint32_t)B->n[1], s1 = (uint32_t)B->rs1;
  L.s1 = s1;
  L.s0 = n1 * s1;
  L.e0 = (uint32_t)B->ctrl_off + ((uint32_t)L.j[0] * n1 + (uint32_t)L.j[1]) * s1 + (uint32_t)L.j[2];
  L.mc = macro_cell(m, B, L.j);
  return L;
}

template <int P, bool MULTI, bool GT = false>
__device__ __forceinline__ Loc locate(const DevModel& m, const SpanRec* __restrict__ R,
                                      const double (&x)[3], const double* __restrict__ EDG) {
  Probe q = probe<MULTI, GT>(m, R, x, EDG);
  return finish(m, R, q);
}

template <int P, bool MULTI, bool GT = false>
__device__ __forceinline__ Loc locate(const DevModel& m, const SpanRec* __restrict__ R,
                                      const double (&x)[3]) {
  return locate<P, MULTI, GT>(m, R, x, m.edges);
}

// Value and world gradient at a located point: the control-row loads are
// issued first, so the basis is computed while they are in flight.
template <int P, Storage S, bool UNIFORM_STRIDES>
__device__ __forceinline__ float4 evaluate(const Loc& L, __amdgpu_buffer_rsrc_t rs,
                                           const float* __restrict__ mats, int stride, int imat) {
  float N[3][P + 1], D[3][P + 1];
#pragma unroll
  for (int a = 0; a < 3; ++a) basis<P>(mats, stride, L.mat[a], imat, L.tau[a], N[a], D[a]);
  float f, fx, fy, fz;
  auto row = [&](int i, int j, float (&v)[P + 1]) {
    uint32_t w[Row<P, S>::kWords];
    if constexpr (UNIFORM_STRIDES)
      Row<P, S>::load(rs, L.e0, (uint32_t)i * L.s0 + (uint32_t)j * L.s1, w);
    else
      Row<P, S>::load(rs, L.e0 + (uint32_t)i * L.s0 + (uint32_t)j * L.s1, 0u, w);
    Row<P, S>::unpack(w, L.e0, v);
  };
  contract_rows<P>(row, N[0], D[0], N[1], D[1], N[2], D[2], f, fx, fy, fz);
  return make_float4(f, fx * L.ds[0], fy * L.ds[1], fz * L.ds[2]);
}

// ------------------------------------------------------------------ K1: points
// Result of point i: (f, df/dx, df/dy, df/dz) as a float4 at out[4 i], or
// (G = false, value-only queries) f alone at out[i]; the gradient terms of
// the contraction and the derivative basis are then dead code.
template <bool G>
__device__ __forceinline__ void put_result(float* __restrict__ out, int64_t i, const float4& e) {
  if constexpr (G)
    reinterpret_cast<float4*>(out)[i] = e;
  else
    out[i] = e.x;
}

template <int P, Storage S, bool MULTI, bool GT = false, bool G = true>
__global__ __launch_bounds__(kBlock) void decode_points_k(DevModel m, const float* __restrict__ xyz,
                                                          int64_t n, float* __restrict__ out,
                                                          int32_t* __restrict__ dbg) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const double x[3] = {(double)xyz[i], (double)xyz[n + i], (double)xyz[2 * n + i]};
  const Loc L = locate<P, MULTI, GT>(m, m.rec, x);
  put_result<G>(out, i, evaluate<P, S, !MULTI>(L, rs, m.mats, m.mat_stride, m.imat));
  if (dbg) reinterpret_cast<int4*>(dbg)[i] = make_int4(L.j[0] + P, L.j[1] + P, L.j[2] + P, L.block);
}

// Workgroup i runs on XCD i % 8: deal contiguous bands of work items to
// XCDs so each XCD's L2 holds what its workgroups touch.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
  const int x = bid & 7, q = bid >> 3;
  const int per = ntiles >> 3, rem = ntiles & 7;
  return x * per + (x < rem ? x : rem) + q;
}

// ------------------------------------------------------------------ K5: sort by (block, tile)
// Multisplit of the points by bucket = (owning block, tile of 2^sort_shift
// spans per axis).  The bucket only orders the work; every point is then
// evaluated by the same exact rules, so the results do not depend on it.
// A histogram pass counts the buckets of large chunks in LDS (two 16-bit
// counters per word) and adds them to the global counts; a one-workgroup
// scan gives each bucket's start and the list of decode items; scatter
// passes recount each chunk, claim a run per key with one global atomic,
// and write the records (x, y, z, input index) into those runs.  With up to
// kOneLevelBuckets buckets one pass writes runs of tens of records; above,
// runs per bucket would be a record or two, which HBM takes as partial-line
// writes, so the points go first to their coarse key (bucket >> fine_shift,
// at most kCoarseBuckets keys) and then, from those coarse runs, to their
// buckets: a chunk of the second pass covers one or two coarse keys, so its
// keys relative to the chunk's first coarse key fit a small LDS table.
constexpr int kFineKeys = 1024;                    // LDS keys of a fine-pass chunk
constexpr int kHistThreads = 1024;                 // histogram workgroup
// Points per thread and chunk of the histogram (a chunk < 65536 points):
// measured best at 63 for single blocks, 16 for multi-block models.
template <bool MULTI>
constexpr int hist_per() { return MULTI ? 16 : 63; }
template <bool MULTI>
constexpr int hist_chunk() { return kHistThreads * hist_per<MULTI>(); }
constexpr int kHistGrid = 2 * 256;                 // two workgroups per CU, each with a range of chunks
constexpr int kScanThreads = 1024;

// Sort tables of a multi-block model in LDS: block edges (FP32), then one
// SortBlk per block; the global copies when the model exceeds the LDS
// budget.
struct SortTabs {
  const SortBlk* blk;
  const float* edges;
};

// LDS bytes of the staged sort tables (0: not staged); the launchers add
// them to the dynamic LDS of the sort kernels.
template <bool MULTI>
__host__ __device__ inline size_t sort_tabs_bytes(const DevModel& m) {
  if (!MULTI) return 0;
  return m.nblocks <= kSortBlkLds && m.n_edges <= kSortEdgesLds
             ? (size_t)m.nblocks * sizeof(SortBlk) + (size_t)((m.n_edges + 3) / 4) * 16
             : 0;
}

// TL (tables in LDS, sort_tabs_bytes() != 0) is a compile-time choice, so
// that the table reads compile to LDS loads rather than generic ones.
template <bool MULTI, bool TL>
__device__ __forceinline__ SortTabs stage_sort_tabs(const DevModel& m, float4* lds) {
  SortTabs t{m.sblk, m.sedges};
  if constexpr (MULTI && TL) {
    SortBlk* lb = reinterpret_cast<SortBlk*>(lds);
    float* le = reinterpret_cast<float*>(lb + m.nblocks);
    for (int q = threadIdx.x; q < m.nblocks * 3; q += blockDim.x)
      reinterpret_cast<float4*>(lb)[q] = reinterpret_cast<const float4*>(m.sblk)[q];
    for (int q = threadIdx.x; q < m.n_edges; q += blockDim.x) le[q] = m.sedges[q];
    t.blk = lb;
    t.edges = le;
    __syncthreads();
  }
  return t;
}

// Bucket of a point.  Single-block models: the tile of the span guesses
// (the exact span or, within rounding of a knot, a neighbour).  Multi-block
// models, in FP32 (the bucket only orders the work): the block from the
// FP32 edges (the exact owner except within FP32 rounding of a face, which
// the decode detects) and the tile of floor((x - lo) * nsp / (hi - lo)).
template <bool MULTI, bool GT>
__device__ __forceinline__ uint32_t sort_bucket(const DevModel& m, const SortTabs& tb,
                                                const float (&x)[3]) {
  int t[3], td[3];
  uint32_t off;
  if constexpr (MULTI) {
    int b[3];
    float xc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float* E = tb.edges + m.edge_off[a];
      const int G = m.grid[a];
      xc[a] = fminf(fmaxf(x[a], E[0]), E[G]);
      int bb = (int)((xc[a] - E[0]) * (float)m.edge_scale[a]);
      bb = bb < 0 ? 0 : (bb > G - 1 ? G - 1 : bb);
      if (bb < G - 1 && E[bb + 1] <= xc[a]) ++bb;
      else if (bb > 0 && E[bb] > xc[a]) --bb;
      b[a] = bb;
    }
    const SortBlk& B = tb.blk[(b[0] * m.grid[1] + b[1]) * m.grid[2] + b[2]];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int nt = B.nt[a];
      const int j = (int)((xc[a] - B.lo[a]) * B.tscale[a]);    // tile of the FP32 span
      t[a] = j < 0 ? 0 : (j > nt - 1 ? nt - 1 : j);
      td[a] = nt;
    }
    off = (uint32_t)B.tile_off;
  } else {
    const DevBlock* __restrict__ B = &m.b0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double xa = (double)x[a];
      const double u = param_of(clampd(xa, m.box_lo[a], m.box_hi[a]), m.box_lo[a], B->inv_ext[a]);
      const int nsp = B->nsp[a], sh = m.sort_shift;
      t[a] = guess_span<GT>(m, B, 0, a, u) >> sh;
      td[a] = (nsp + (1 << sh) - 1) >> sh;
    }
    off = 0;
  }
  return off + (uint32_t)((t[0] * td[1] + t[1]) * td[2] + t[2]);
}

__global__ __launch_bounds__(kBlock) void fill_u32_k(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Bucket counts of an equal range of points per workgroup, taken in chunks
// of at most hist_chunk() points: 16-bit counters, two per LDS word
// (bucket b in the half b & 1 of word b >> 1), added to the global counts
// at the end.  Before each later chunk a counter above kSafe (which the
// chunk could take past 65535) is moved to the global counts first.
// Few workgroups, each with many points, keep the final global additions
// (one per bucket and workgroup) few.  Dynamic LDS: the sort tables, then
// the counters.
template <bool MULTI, bool GT, bool TL>
__global__ __launch_bounds__(kHistThreads, MULTI ? 8 : 1) void sort_hist_k(DevModel m, SortArgs sa) {
  // Multi-block models hold up to kMaxBuckets 16-bit counters (64 KB of
  // LDS), so two workgroups fit a CU only at eight waves per SIMD, i.e. at
  // most 64 registers: two points per step there, four otherwise.
  constexpr int kHistIlp = MULTI ? 2 : 4;
  constexpr int kHistPer = hist_per<MULTI>(), kHistChunk = hist_chunk<MULTI>();
  constexpr uint32_t kSafe = 65535u - (uint32_t)kHistChunk;
  extern __shared__ float4 sdyn[];
  const SortTabs tb = stage_sort_tabs<MULTI, TL>(m, sdyn);
  uint32_t* h = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(sdyn) +
                                            (TL ? sort_tabs_bytes<MULTI>(m) : 0));
  const int nw = (sa.nb + 1) >> 1;
  for (int w = threadIdx.x; w < nw; w += kHistThreads) h[w] = 0u;
  __syncthreads();
  // the workgroup's range [r0, r1): a multiple of kHistThreads points
  const int64_t per = ((sa.n + gridDim.x - 1) / gridDim.x + kHistThreads - 1) / kHistThreads * kHistThreads;
  const int64_t r0 = min(sa.n, (int64_t)blockIdx.x * per), r1 = min(sa.n, r0 + per);
  for (int64_t c0 = r0; c0 < r1; c0 += kHistChunk) {
    if (c0 != r0) {
      // the previous chunk's LDS additions must have landed before the
      // counters are read: the compiler leaves this barrier (reached over
      // the loop's back edge) without that wait, so it is made explicit
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      __syncthreads();
      for (int w = threadIdx.x; w < nw; w += kHistThreads) {
        const uint32_t v = h[w], lo = v & 0xFFFFu, hi = v >> 16;
        if (lo > kSafe || hi > kSafe) {
          if (lo > kSafe) atomicAdd(sa.hist + 2 * w, lo);
          if (hi > kSafe) atomicAdd(sa.hist + 2 * w + 1, hi);
          h[w] = (lo > kSafe ? 0u : lo) | ((hi > kSafe ? 0u : hi) << 16);
        }
      }
      __syncthreads();
    }
    // kHistIlp independent points per step keep several bucket computations
    // (chains of dependent LDS loads) in flight per thread.  The points of
    // the next step are loaded before this step's bucket ids are stored: a
    // wait for loads also waits for the stores issued before them
    auto load = [&](int q, float (&x)[kHistIlp][3]) {
#pragma unroll
      for (int u = 0; u < kHistIlp; ++u) {
        const int64_t i = c0 + (int64_t)(q + u) * kHistThreads + threadIdx.x;
        const int64_t ic = q + u < kHistPer && i < r1 ? i : 0;
        x[u][0] = sa.xyz[ic];
        x[u][1] = sa.xyz[sa.n + ic];
        x[u][2] = sa.xyz[2 * sa.n + ic];
      }
    };
    float x[kHistIlp][3];
    load(0, x);
    for (int q = 0; q < kHistPer; q += kHistIlp) {
      uint32_t b[kHistIlp];
#pragma unroll
      for (int u = 0; u < kHistIlp; ++u) b[u] = sort_bucket<MULTI, GT>(m, tb, x[u]);
      if (q + kHistIlp < kHistPer) load(q + kHistIlp, x);
#pragma unroll
      for (int u = 0; u < kHistIlp; ++u) {
        const int64_t i = c0 + (int64_t)(q + u) * kHistThreads + threadIdx.x;
        if (q + u < kHistPer && i < r1) {
          atomicAdd(h + (b[u] >> 1), 1u << ((b[u] & 1u) * 16u));
          if (sa.bkt) sa.bkt[i] = (uint16_t)b[u];
        }
      }
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nw; w += kHistThreads) {
    const uint32_t v = h[w];
    if (v & 0xFFFFu) atomicAdd(sa.hist + 2 * w, v & 0xFFFFu);
    if (v >> 16) atomicAdd(sa.hist + 2 * w + 1, v >> 16);
  }
}

// Exclusive scan over the workgroup of one value per thread (kScanThreads
// threads); returns the thread's exclusive prefix, the total in *tot.
// wsum: kScanThreads / kWave words.
__device__ __forceinline__ uint32_t block_scan(uint32_t s, uint32_t* wsum, uint32_t* tot) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t inc = s;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  __syncthreads();
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t run = inc - s, all = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if (w < wave) run += wsum[w];
    all += wsum[w];
  }
  *tot = all;
  return run;
}

// Decode parts of a bucket of c points: ceil(c / kTilePoints).
__device__ __forceinline__ uint32_t n_parts(uint32_t c) { return (c + kTilePoints - 1) / kTilePoints; }

// One workgroup: exclusive scan of the bucket counts (start[nb] = n), reset
// of the cursors, and the list of decode items (bucket, part) in bucket
// order; rounds of kScanThreads buckets, one per thread, with the running
// totals carried from round to round.
__global__ __launch_bounds__(kScanThreads) void sort_scan_k(SortArgs sa) {
  __shared__ uint32_t wsum[kScanThreads / kWave];
  uint32_t run0 = 0, irun0 = 0;
  for (int r0 = 0; r0 < sa.nb; r0 += kScanThreads) {
    const int b = r0 + threadIdx.x;
    const uint32_t v = b < sa.nb ? sa.hist[b] : 0u;
    const uint32_t np = n_parts(v);
    uint32_t tot, itot;
    const uint32_t run = run0 + block_scan(v, wsum, &tot);
    const uint32_t irun = irun0 + block_scan(np, wsum, &itot);
    if (b < sa.nb) {
      sa.start[b] = run;
      sa.cursor[b] = 0u;
      for (uint32_t u = 0; u < np; ++u) sa.items[irun + u] = make_int2(b, (int)u);
    }
    run0 += tot;
    irun0 += itot;
    __syncthreads();                               // wsum reused by the next round
  }
  if (threadIdx.x == 0) {
    *sa.n_items = (int32_t)irun0;
    sa.start[sa.nb] = (uint32_t)sa.n;
  }
  if (sa.tmp && threadIdx.x < kCoarseBuckets) sa.ccursor[threadIdx.x * kCursorStride] = 0u;
}

// Record i of the pass input: the points in input order, or (FROM_TMP) the
// records of the coarse pass.  BR: the fourth word of a point's record is
// its bucket (from sa.bkt) rather than its input index.
template <bool FROM_TMP, bool BR>
__device__ __forceinline__ float4 sort_input(const SortArgs& sa, int64_t i) {
  if constexpr (FROM_TMP)
    return sa.tmp[i];
  else
    return make_float4(sa.xyz[i], sa.xyz[sa.n + i], sa.xyz[2 * sa.n + i],
                       __uint_as_float(BR ? (uint32_t)sa.bkt[i] : (uint32_t)i));
}

// Exclusive scan over n <= 4 * kBlock LDS counters by the workgroup (kBlock
// threads): v[k] becomes the sum of v[0..k-1], *total the sum of all.
// wsum: kBlock / kWave words.
__device__ __forceinline__ void lds_scan(uint32_t* v, int n, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int k0 = threadIdx.x * 4;
  uint32_t a[4], s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = k0 + q < n ? v[k0 + q] : 0u;
    s += a[q];
  }
  uint32_t inc = s;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t run = inc - s;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  if (threadIdx.x == kBlock - 1) *total = run + s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (k0 + q < n) v[k0 + q] = run;
    run += a[q];
  }
  __syncthreads();
}

// Scatter pass over one chunk of kScatterChunk records.  Each record's key
// and rank within the chunk come from LDS counters; the chunk is then
// ordered by key in LDS and written out by consecutive threads to
// consecutive positions of each key's run (one run per key and chunk,
// claimed with one global atomic), so the writes reach memory as whole
// lines.
//  kOne:    key = bucket, input order, runs from sa.cursor into sa.rec;
//  kCoarse: key = bucket >> fine_shift, input order, runs from sa.ccursor
//           into sa.tmp;
//  kFine:   key = bucket, from sa.tmp (coarse order), runs from sa.cursor
//           into sa.rec; the LDS counters cover kFineKeys keys from the
//           first coarse key of the chunk on (at least two coarse keys); a
//           record beyond them claims its slot with its own global atomic
//           and is written directly (chunks spanning several short coarse
//           runs only).
constexpr int kOne = 0, kCoarse = 1, kFine = 2;
constexpr int kScatterPer = 8;
constexpr int kScatterChunk = kBlock * kScatterPer;

// The pass input records of the chunk at c0 held by this thread (record
// l = q * kBlock + threadIdx.x in in[q]; zeros past the end).
template <int MODE, bool BR>
__device__ __forceinline__ void load_chunk(const SortArgs& sa, int64_t c0, float4 (&in)[kScatterPer]) {
  const int64_t cn = min((int64_t)kScatterChunk, sa.n - c0);
#pragma unroll
  for (int q = 0; q < kScatterPer; ++q) {
    const int l = q * kBlock + threadIdx.x;
    in[q] = l < cn ? sort_input<MODE == kFine, BR>(sa, c0 + l) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// One chunk of the scatter pass (see sort_scatter_k), its records in in[].
// BR (two levels with sa.tpos and sa.bkt): the bucket is the fourth word
// of the pass input records; the coarse pass keeps it there, the bucket
// pass replaces it with the record's position in the coarse order.
template <bool MULTI, int MODE, bool GT, int kKeys, bool BR>
__device__ __forceinline__ void scatter_chunk(const DevModel& m, const SortArgs& sa, const SortTabs& tb,
                                              int64_t c0, const float4 (&in)[kScatterPer], uint32_t* h,
                                              uint32_t* gbase, float4* recs, uint16_t* keyof,
                                              uint32_t* wsum, uint32_t* s_key0, uint32_t* s_staged) {
  constexpr int PER = kScatterPer;
  const int cn = (int)min((int64_t)kScatterChunk, sa.n - c0);
  if constexpr (MODE == kFine) {
    if (threadIdx.x == 0) {
      const float4 r = sa.tmp[c0];
      const float x[3] = {r.x, r.y, r.z};
      const uint32_t b0 = BR ? __float_as_uint(r.w) : sort_bucket<MULTI, GT>(m, tb, x);
      *s_key0 = (b0 >> sa.fine_shift) << sa.fine_shift;
    }
  }
  const int nk = MODE == kCoarse ? ((sa.nb + (1 << sa.fine_shift) - 1) >> sa.fine_shift)
                                 : (MODE == kOne ? sa.nb : kFineKeys);
  for (int b = threadIdx.x; b < nk; b += kBlock) h[b] = 0u;
  __syncthreads();
  uint32_t key0 = 0;
  if constexpr (MODE == kFine) key0 = *s_key0;
  float4 rec[PER];
  uint32_t key[PER], rank[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int l = q * kBlock + threadIdx.x;
    key[q] = 0xFFFFFFFFu;
    if (l < cn) {
      rec[q] = in[q];
      const float x[3] = {rec[q].x, rec[q].y, rec[q].z};
      const uint32_t b = BR ? __float_as_uint(rec[q].w) : sort_bucket<MULTI, GT>(m, tb, x);
      if constexpr (MODE == kFine)
        if (sa.tpos) rec[q].w = __uint_as_float((uint32_t)(c0 + l));   // position in tmp
      if constexpr (MODE == kCoarse) {
        key[q] = b >> sa.fine_shift;
        rank[q] = atomicAdd(h + key[q], 1u);
      } else if constexpr (MODE == kOne) {
        key[q] = b;
        rank[q] = atomicAdd(h + key[q], 1u);
      } else {
        const uint32_t k = b - key0;              // b >= key0: coarse runs are in key order
        if (k < (uint32_t)kFineKeys) {
          key[q] = k;
          rank[q] = atomicAdd(h + k, 1u);
        } else {                                  // beyond the table: own slot, written now
          key[q] = 0xFFFFFFFEu;
          const uint32_t pos = sa.start[b] + atomicAdd(sa.cursor + b, 1u);
          if ((int64_t)pos < sa.n) sa.rec[pos] = rec[q];
        }
      }
    }
  }
  __syncthreads();
  // one run per key and chunk
  for (int b = threadIdx.x; b < nk; b += kBlock)
    if (h[b]) {
      if constexpr (MODE == kCoarse)
        gbase[b] = sa.start[b << sa.fine_shift] + atomicAdd(sa.ccursor + b * kCursorStride, h[b]);
      else
        gbase[b] = sa.start[key0 + b] + atomicAdd(sa.cursor + key0 + b, h[b]);
    }
  lds_scan(h, nk, wsum, s_staged);             // h: chunk-local start of each key
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (key[q] >= 0xFFFFFFFEu) continue;
    const uint32_t sl = h[key[q]] + rank[q];
    recs[sl] = rec[q];
    keyof[sl] = (uint16_t)key[q];
    if constexpr (MODE == kCoarse)
      if (sa.tpos) sa.tpos[c0 + q * kBlock + threadIdx.x] = gbase[key[q]] + rank[q];
  }
  __syncthreads();
  float4* dst = MODE == kCoarse ? sa.tmp : sa.rec;
  const int staged = (int)*s_staged;          // cn less the records written directly
  for (int sl = threadIdx.x; sl < staged; sl += kBlock) {
    const uint32_t k = keyof[sl];
    const uint32_t pos = gbase[k] + ((uint32_t)sl - h[k]);
    if ((int64_t)pos < sa.n) dst[pos] = recs[sl];
  }
  __syncthreads();                             // LDS reused by the next chunk
}

// The workgroups loop over chunks (see the bands below), so the sort tables
// are staged once per workgroup rather than once per chunk; the records of
// a workgroup's next chunk are loaded while it orders and writes the
// current one.
template <bool MULTI, int MODE, bool GT, bool TL, bool BR = false>
__global__ __launch_bounds__(kBlock) void sort_scatter_k(DevModel m, SortArgs sa) {
  constexpr int kKeys = MODE == kCoarse ? kCoarseBuckets : (MODE == kOne ? kOneLevelBuckets : kFineKeys);
  static_assert(kKeys <= 4 * kBlock, "lds_scan covers 4 keys per thread");
  __shared__ uint32_t h[kKeys];          // counts, then the chunk-local start of each key
  __shared__ uint32_t gbase[kKeys];      // global start of each key's run
  __shared__ float4 recs[kScatterChunk]; // the chunk in key order
  __shared__ uint16_t keyof[kScatterChunk];
  __shared__ uint32_t wsum[kBlock / kWave];
  __shared__ uint32_t s_key0, s_staged;
  extern __shared__ float4 sdyn[];
  const SortTabs tb = stage_sort_tabs<MULTI, TL>(m, sdyn);
  // the chunks in eight contiguous bands, band x to the workgroups of XCD x
  // (workgroups go to the XCDs round-robin; the grid is a multiple of 8):
  // the runs that one key's chunks append to are then written through one
  // L2, where their lines fill up before they are written back
  const int64_t nch = (sa.n + kScatterChunk - 1) / kScatterChunk;
  const int xcd = (int)(blockIdx.x & 7u), nx = (int)(gridDim.x >> 3);
  const int64_t hi = nch * (xcd + 1) / 8;
  int64_t c = nch * xcd / 8 + (int64_t)(blockIdx.x >> 3);
  float4 cur[kScatterPer];
  load_chunk<MODE, BR>(sa, c < hi ? c * kScatterChunk : sa.n, cur);
  for (; c < hi; c += nx) {
    float4 nxt[kScatterPer];
    load_chunk<MODE, BR>(sa, c + nx < hi ? (c + nx) * kScatterChunk : sa.n, nxt);
    scatter_chunk<MULTI, MODE, GT, kKeys, BR>(m, sa, tb, c * kScatterChunk, cur, h, gbase, recs, keyof,
                                              wsum, &s_key0, &s_staged);
#pragma unroll
    for (int q = 0; q < kScatterPer; ++q) cur[q] = nxt[q];
  }
}

// One stored control point, converted to FP32 as the row loaders do.
template <Storage S>
__device__ __forceinline__ float load_one(__amdgpu_buffer_rsrc_t rs, uint32_t e) {
  if constexpr (S == Storage::F32) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, e * 4u, 0u, 0));
  } else {
    const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(rs, e * 2u, 0u, 0);
    if constexpr (S == Storage::BF16)
      return __uint_as_float((uint32_t)h << 16);
    else
      return __half2float(__ushort_as_half(h));
  }
}

// Value and world gradient with the control rows read from an LDS window:
// Wp points at P[i0][j0][k0] of the window, rows at + i*sw0 + j*sw1.
template <int P>
__device__ __forceinline__ float4 evaluate_lds(const Loc& L, const float* Wp, int sw0, int sw1,
                                               const float* __restrict__ mats, int stride,
                                               int imat) {
  float N[3][P + 1], D[3][P + 1];
#pragma unroll
  for (int a = 0; a < 3; ++a) basis<P>(mats, stride, L.mat[a], imat, L.tau[a], N[a], D[a]);
  float f, fx, fy, fz;
  auto row = [&](int i, int j, float (&v)[P + 1]) {
    const float* r = Wp + i * sw0 + j * sw1;
#pragma unroll
    for (int k = 0; k <= P; ++k) v[k] = r[k];
  };
  contract_rows<P>(row, N[0], D[0], N[1], D[1], N[2], D[2], f, fx, fy, fz);
  return make_float4(f, fx * L.ds[0], fy * L.ds[1], fz * L.ds[2]);
}

// A point of a known block B (the sort placed it in one of B's buckets by
// the block-owner rule, the one probe() applies): the parameter map and the
// span guesses with their records, as probe() computes them for B.  TR:
// the records of the tile's spans o[a] .. o[a] + ns[a] - 1 per axis (axis a
// from toff[a] on), or null; a guess outside them reads R.
template <bool GT, int NT>
__device__ __forceinline__ Probe probe_block(const DevModel& m, const SpanRec* __restrict__ R,
                                             const double (&x)[3], const DevBlock* __restrict__ B,
                                             int block, const SpanRec (&TR)[NT], bool tr_ok,
                                             const int (&o)[3], const int (&ns)[3],
                                             const int (&toff)[3]) {
  Probe q;
  q.B = B;
  q.block = block;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.b[a] = 0;
    q.u[a] = param_of(clampd(x[a], m.box_lo[a], m.box_hi[a]), B->lo[a], B->inv_ext[a]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.j[a] = guess_span<GT>(m, B, block, a, q.u[a]);
    const int jj = q.j[a] - o[a];
    if (tr_ok && jj >= 0 && jj < ns[a])
      q.rec[a] = TR[toff[a] + jj];
    else
      q.rec[a] = R[B->rec_off[a] + q.j[a]];
  }
  return q;
}

constexpr int kTileRecs = 96;      // span records of a tile staged for multi-block decodes

// A record read by every lane at the same address, kept as wave-uniform
// values (scalar registers).
template <class T>
__device__ __forceinline__ T uniform_copy(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T b;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&b);
#pragma unroll
  for (int q = 0; q < (int)(sizeof(T) / 4); ++q) dst[q] = __builtin_amdgcn_readfirstlane(src[q]);
  return b;
}

// Basis tables held in LDS by the kernels that do not stage them with the
// span records: at most kMatsLds floats (clamped uniform knots share a few
// span shapes); models with more take kernels that read the global pool.
// The tables are staged before the kernels' own first barrier.
constexpr int kMatsLds = 1024;

// Copy of n float4 from global memory into LDS by a whole workgroup, four
// loads per thread in flight before their LDS writes (a loop that writes
// each value as it arrives waits out one memory latency per value).  Slots
// past the end repeat the last element, which lands where its own copy
// does, so every load and write is unconditional.
__device__ __forceinline__ void stage_lds(float4* dst, const float4* __restrict__ src, int n) {
  constexpr int U = 4;
  for (int q0 = threadIdx.x; q0 < n; q0 += U * kBlock) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[min(q0 + u * kBlock, n - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) dst[min(q0 + u * kBlock, n - 1)] = v[u];
  }
}

// Decode in sorted order, one item (a bucket, or an equal part of a bucket
// of more than kTilePoints points) per workgroup; results go to the input
// positions.  The bucket's window of control points (the tile's spans plus
// p per axis) is staged in LDS once (when it holds at most win_cap values);
// a point whose exact spans fall outside the window reads its rows from
// global memory.  Both paths sum in the same order.  LDSREC: the span
// records and basis tables of a single-block model are staged too, ahead of
// the window.  Multi-block models: every point of the bucket lies in the
// bucket's block, whose record the workgroup reads as uniform data.  For
// those at degree <= 3 the launch bounds ask for four waves per SIMD: left
// alone the compiler takes 133 registers (three waves) where 105 suffice.
template <int P, Storage S, bool MULTI, bool LDSREC, bool GT = false, bool G = true>
__global__ __launch_bounds__(kBlock, (MULTI && P <= 3) ? 4 : 1) void decode_tiles_k(DevModel m, SortArgs sa, int win_cap,
                                                         float* __restrict__ out,
                                                         int32_t* __restrict__ dbg) {
  extern __shared__ float4 dyn[];
  __shared__ float4 lmats[LDSREC ? 1 : kMatsLds / 4];
  const int item = blockIdx.x;
  if (item >= *sa.n_items) return;                 // whole workgroup
  const SpanRec* R = m.rec;
  const float* MT = m.mats;
  float* W = reinterpret_cast<float*>(dyn);
  if constexpr (LDSREC) {
    SpanRec* lr = reinterpret_cast<SpanRec*>(dyn);
    float* lm = reinterpret_cast<float*>(lr + m.n_rec);
    stage_lds(reinterpret_cast<float4*>(lr), reinterpret_cast<const float4*>(m.rec), m.n_rec * 2);
    stage_lds(reinterpret_cast<float4*>(lm), reinterpret_cast<const float4*>(m.mats),
              m.n_mats * m.mat_stride / 4);
    R = lr;
    MT = lm;
    W = lm + m.n_mats * m.mat_stride;
  } else {
    // the launcher sends models whose tables exceed kMatsLds floats to
    // decode_sorted_k, so that these reads are always LDS loads
    stage_lds(lmats, reinterpret_cast<const float4*>(m.mats), m.n_mats * m.mat_stride / 4);
    MT = reinterpret_cast<const float*>(lmats);
  }
  const int2 it = uniform_copy(sa.items + item);
  const int b = it.x;
  const uint32_t b0 = __builtin_amdgcn_readfirstlane(sa.start[b]);
  const uint32_t bcnt = __builtin_amdgcn_readfirstlane(sa.start[b + 1]) - b0, np = n_parts(bcnt);
  const uint32_t s0 = b0 + (uint32_t)(((uint64_t)bcnt * (uint32_t)it.y) / np);
  const uint32_t s1 = b0 + (uint32_t)(((uint64_t)bcnt * (uint32_t)(it.y + 1)) / np);
  const BucketWin bw = uniform_copy(m.bwin + b);
  const int w12 = bw.w[1] * bw.w[2];
  const int wn = bw.w[0] * w12;
  const bool staged = wn <= win_cap;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  // multi-block models: the bucket's block record as uniform values (the
  // block is the same for the whole workgroup), and the span records of
  // the tile per axis in LDS
  DevBlock Bu;
  int bq[3] = {0, 0, 0};
  double be0[3] = {0.0, 0.0, 0.0}, be1[3] = {0.0, 0.0, 0.0};
  if constexpr (MULTI) {
    Bu = uniform_copy(m.blocks + bw.block);
    // the block's grid coordinates and bracketing edges, for the exact
    // owner check of each point (the bucket was found in FP32)
    bq[2] = bw.block % m.grid[2];
    bq[1] = (bw.block / m.grid[2]) % m.grid[1];
    bq[0] = bw.block / (m.grid[2] * m.grid[1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      be0[a] = uniform_copy(m.edges + m.edge_off[a] + bq[a]);
      be1[a] = uniform_copy(m.edges + m.edge_off[a] + bq[a] + 1);
    }
  }
  const DevBlock* __restrict__ B = MULTI ? &Bu : &m.b0;
  __shared__ SpanRec trec[MULTI ? kTileRecs : 1];
  int ns[3], toff[3];
  bool tr_ok = false;
  if constexpr (MULTI) {
    int tot = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ns[a] = bw.w[a] - P;
      toff[a] = tot;
      tot += ns[a];
    }
    tr_ok = tot <= kTileRecs;
    if (tr_ok) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        for (int q = threadIdx.x; q < ns[a]; q += kBlock)
          trec[toff[a] + q] = m.rec[B->rec_off[a] + bw.o[a] + q];
    }
  }
  if (staged) {
    // lanes cover rpi whole rows of the window per pass (k = lane % w2);
    // the row index (i, j) of each lane advances without divisions
    const uint32_t n1 = (uint32_t)B->n[1], rs1 = (uint32_t)B->rs1;
    const int w1 = bw.w[1], w2 = bw.w[2], rows = bw.w[0] * w1;
    if (w2 <= kWave) {
      // U rows per lane per pass, their loads in flight together.  A slot
      // past the last row reads and writes the last row's value, and a lane
      // past rpi rows (sub >= rpi) reads and writes a row another wave
      // covers: duplicate writes of equal values, so none is conditional.
      constexpr int U = 4;
      const int rpi = kWave / w2, lane = threadIdx.x & (kWave - 1);
      const int sub = lane / w2, k = lane - sub * w2;
      const int step = rpi * (kBlock / kWave);
      int row = (threadIdx.x / kWave) * rpi + sub;
      int i = row / w1, j = row - i * w1;
      const int di = step / w1, dj = step - di * w1;
      for (; row < rows; row += U * step) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = row + u * step < rows;
          const uint32_t e = (uint32_t)B->ctrl_off +
                             ((uint32_t)(bw.o[0] + (ok ? i : bw.w[0] - 1)) * n1 +
                              (uint32_t)(bw.o[1] + (ok ? j : w1 - 1))) * rs1 +
                             (uint32_t)(bw.o[2] + k);
          v[u] = load_one<S>(rs, e);
          i += di;
          j += dj;
          if (j >= w1) {
            j -= w1;
            ++i;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) W[min(row + u * step, rows - 1) * w2 + k] = v[u];
      }
    } else {
      for (int q = threadIdx.x; q < wn; q += kBlock) {
        const int i = q / w12, r = q - i * w12, j = r / w2, k = r - j * w2;
        const uint32_t e = (uint32_t)B->ctrl_off +
                           ((uint32_t)(bw.o[0] + i) * n1 + (uint32_t)(bw.o[1] + j)) * rs1 +
                           (uint32_t)(bw.o[2] + k);
        W[q] = load_one<S>(rs, e);
      }
    }
  }
  __syncthreads();                 // window and tile records staged
  if (s0 >= s1) return;
  // Loads and stores share one completion counter here, and a wait for a
  // load with a store in flight waits for everything.  So each step first
  // takes its record (loaded one step earlier; the empty asm is the point
  // where the compiler waits for it, and no memory access moves above it),
  // then stores the previous step's result and loads the next record: the
  // one wait of the next step finds that store and load a whole step old.
  constexpr uint32_t kNone = 0xffffffffu;
  uint32_t pi = kNone;             // input position of the pending result
  float4 pres = make_float4(0.f, 0.f, 0.f, 0.f);
  const f32x4* __restrict__ rec4 = reinterpret_cast<const f32x4*>(sa.rec);
  uint32_t t = s0 + threadIdx.x;
  // each record is read once: streaming loads
  f32x4 q = __builtin_nontemporal_load(rec4 + min(t, s1 - 1));
  for (; t < s1; t += kBlock) {
    asm volatile("" : "+v"(q) : : "memory");
    const double x[3] = {(double)q.x, (double)q.y, (double)q.z};
    const uint32_t i = __float_as_uint(q.w);
    if (pi != kNone) put_result<G>(out, pi, pres);
    pi = kNone;
    q = __builtin_nontemporal_load(rec4 + min(t + kBlock, s1 - 1));
    Loc L;
    if constexpr (MULTI) {
      bool own = true;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        own &= owner_ok(m.grid[a], clampd(x[a], m.box_lo[a], m.box_hi[a]), bq[a], be0[a], be1[a]);
      if (own) {
        Probe pr = probe_block<GT>(m, R, x, B, bw.block, trec, tr_ok, bw.o, ns, toff);
        L = finish(m, R, pr);
      } else {                         // within FP32 rounding of a block face
        L = locate<P, true, GT>(m, R, x);
      }
    } else {
      L = locate<P, false, GT>(m, R, x);
    }
    if ((int64_t)i >= sa.n) continue;
    int d[3];
    bool in = staged && L.block == bw.block;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d[a] = L.j[a] - bw.o[a];
      in = in && d[a] >= 0 && d[a] <= bw.w[a] - 1 - P;
    }
    float4 res;
    if (in)
      res = evaluate_lds<P>(L, W + (d[0] * bw.w[1] + d[1]) * bw.w[2] + d[2], w12, bw.w[2], MT,
                            m.mat_stride, m.imat);
    else
      res = evaluate<P, S, !MULTI>(L, rs, MT, m.mat_stride, m.imat);
    pres = res;
    pi = i;
    if (dbg) reinterpret_cast<int4*>(dbg)[i] = make_int4(L.j[0] + P, L.j[1] + P, L.j[2] + P, L.block);
  }
  if (pi != kNone) put_result<G>(out, pi, pres);
}

// Sorted decode for models whose bucket windows exceed the LDS budget: one
// point per thread over the sorted records (workgroup ranges dealt to XCDs
// in contiguous bands), rows from global memory.
template <int P, Storage S, bool MULTI, bool GT = false, bool G = true>
__global__ __launch_bounds__(kBlock) void decode_sorted_k(DevModel m, SortArgs sa,
                                                          float* __restrict__ out,
                                                          int32_t* __restrict__ dbg) {
  const int nchunks = (int)((sa.n + kBlock - 1) / kBlock);
  const int64_t t = (int64_t)xcd_tile(blockIdx.x, nchunks) * kBlock + threadIdx.x;
  if (t >= sa.n) return;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const float4 q = sa.rec[t];
  const double x[3] = {(double)q.x, (double)q.y, (double)q.z};
  const Loc L = locate<P, MULTI, GT>(m, m.rec, x);
  const uint32_t i = __float_as_uint(q.w);
  if ((int64_t)i >= sa.n) return;
  put_result<G>(out, i, evaluate<P, S, !MULTI>(L, rs, m.mats, m.mat_stride, m.imat));
  if (dbg) reinterpret_cast<int4*>(dbg)[i] = make_int4(L.j[0] + P, L.j[1] + P, L.j[2] + P, L.block);
}

// ------------------------------------------------------------------ K3: grid
// One wave = 64 consecutive entries c of axis 2 for one entry b of axis 1
// and a run of up to ga.ta entries a of axis 0.  The axis-0 bases of the
// run are computed once per workgroup into LDS.  Along the run the wave
// keeps a window Y[r] (r = 0..P) of axis-2/axis-1 partial sums for control
// rows i = j_a + r, sliding it when the axis-0 span advances by one.
template <int P>
struct ABasis {
  float N[P + 1];
  float D[P + 1];
  float ds;
  int j;
};

constexpr int kGridTA = 64;

template <int P>
__device__ __forceinline__ void axis_basis(const DevModel& m, int a, double uraw, float (&N)[P + 1],
                                           float (&D)[P + 1], float& ds, int& j) {
  const double u = clampd(uraw, 0.0, 1.0);
  SpanRec rec;
  j = locate_span(m.rec + m.b0.rec_off[a], m.b0.nsp[a], u, rec);
  Table<P> c;
  load_table<P>(m.mats + rec.mat * m.mat_stride, c);
  horner<P>(c, local_tau(rec, u), N, D);
  ds = rec.dscale;
}

template <int P, Storage S, bool G = true>
__global__ __launch_bounds__(kBlock) void decode_grid_k(DevModel m, GridArgs ga) {
  __shared__ ABasis<P> sa[kGridTA];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int a0 = blockIdx.z * ga.ta;
  const int na = min(ga.ta, ga.res[0] - a0);
  for (int t = threadIdx.x; t < na; t += kBlock) {
    ABasis<P> ab;
    axis_basis<P>(m, 0, ga.axis[0][a0 + t], ab.N, ab.D, ab.ds, ab.j);
    sa[t] = ab;
    if (ga.spans && blockIdx.x == 0 && blockIdx.y == 0) ga.spans[a0 + t] = ab.j + P;
  }
  __syncthreads();
  const int b = blockIdx.y * (kBlock / kWave) + wave;
  if (b >= ga.res[1]) return;                       // uniform per wave
  const int c = blockIdx.x * kWave + lane;
  const bool cvalid = c < ga.res[2];
  const int cc = cvalid ? c : ga.res[2] - 1;
  float Ny[P + 1], Dy[P + 1], Nz[P + 1], Dz[P + 1], dsy, dsz;
  int jy, jz;
  axis_basis<P>(m, 1, ga.axis[1][b], Ny, Dy, dsy, jy);
  axis_basis<P>(m, 2, ga.axis[2][cc], Nz, Dz, dsz, jz);
  jy = __builtin_amdgcn_readfirstlane(jy);          // b is uniform across the wave
  if (ga.spans) {
    if (blockIdx.x == 0 && blockIdx.z == 0 && lane == 0) ga.spans[ga.res[0] + b] = jy + P;
    if (blockIdx.y == 0 && blockIdx.z == 0 && wave == 0 && cvalid)
      ga.spans[ga.res[0] + ga.res[1] + c] = jz + P;
  }
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const uint32_t n1 = (uint32_t)m.b0.n[1], s1 = (uint32_t)m.b0.rs1;
  const uint32_t ez = (uint32_t)jz;                 // per-lane element offset along axis 2

  // Y/YY/YZ partial sums of control row i over axes 2 and 1.
  auto row = [&](int i, float& y, float& yy, float& yz) {
    y = yy = yz = 0.f;
#pragma unroll
    for (int jj = 0; jj <= P; ++jj) {
      float v[P + 1];
      uint32_t w[Row<P, S>::kWords];
      const uint32_t es = ((uint32_t)i * n1 + (uint32_t)(jy + jj)) * s1;
      Row<P, S>::load(rs, ez, es, w);
      Row<P, S>::unpack(w, ez, v);
      float z = 0.f, zd = 0.f;
#pragma unroll
      for (int k = 0; k <= P; ++k) {
        z = fmaf(Nz[k], v[k], z);
        zd = fmaf(Dz[k], v[k], zd);
      }
      y = fmaf(Ny[jj], z, y);
      yy = fmaf(Dy[jj], z, yy);
      yz = fmaf(Ny[jj], zd, yz);
    }
  };

  float Y[P + 1], YY[P + 1], YZ[P + 1];
  int wj = -(1 << 30);
  const int64_t plane = (int64_t)ga.res[1] * ga.res[2];
  for (int t = 0; t < na; ++t) {
    const int ja = __builtin_amdgcn_readfirstlane(sa[t].j);
    if (ja != wj) {
      if (ja == wj + 1) {
#pragma unroll
        for (int r = 0; r < P; ++r) { Y[r] = Y[r + 1]; YY[r] = YY[r + 1]; YZ[r] = YZ[r + 1]; }
        row(ja + P, Y[P], YY[P], YZ[P]);
      } else {
#pragma unroll
        for (int r = 0; r <= P; ++r) row(ja + r, Y[r], YY[r], YZ[r]);
      }
      wj = ja;
    }
    float f = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
    for (int r = 0; r <= P; ++r) {
      const float nx = sa[t].N[r], dx = sa[t].D[r];
      f = fmaf(nx, Y[r], f);
      fx = fmaf(dx, Y[r], fx);
      fy = fmaf(nx, YY[r], fy);
      fz = fmaf(nx, YZ[r], fz);
    }
    // whole lines, written once: streaming stores
    const int64_t o = (int64_t)(a0 + t) * plane + (int64_t)b * ga.res[2] + c;
    if (cvalid) {
      if constexpr (G)
        store_stream(reinterpret_cast<float4*>(ga.out) + o, make_float4(f, fx * sa[t].ds, fy * dsy, fz * dsz));
      else
        __builtin_nontemporal_store(f, ga.out + o);
    }
  }
}

// ------------------------------------------------------------------ K4: render
// One ray per lane; a workgroup covers a 16x16 pixel tile (four 8x8 waves).
// The cost of a tile follows the image content (rays that miss the volume
// or cross only transparent cells are cheap), so tiles are dealt to the
// XCDs by interleaved tile rows (see frame_tile) rather than in contiguous
// bands, which left the XCDs holding the frame's edges idle.
constexpr int kTile = 16;


struct Ray {
  double o[3], d[3];
  double t_near;
  int K;
};

__device__ __forceinline__ Ray make_ray_box(const double (&blo)[3], const double (&bhi)[3],
                                            const RenderArgs& r, int i, int j) {
#pragma clang fp contract(off)
  Ray ray;
  const double px = (double)(2 * i + 1 - r.w) * r.sx;
  const double py = (double)(r.h - 2 * j - 1) * r.sy;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (r.kind == 0) {
      ray.o[a] = (r.eye[a] + px * r.right[a]) + py * r.up[a];
      ray.d[a] = r.fwd[a];
    } else {
      ray.o[a] = r.eye[a];
      ray.d[a] = (r.fwd[a] + px * r.right[a]) + py * r.up[a];
    }
  }
  double tn = 0.0, tf = __builtin_inf();
  bool miss = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (ray.d[a] == 0.0) {
      miss |= (ray.o[a] < blo[a]) || (ray.o[a] > bhi[a]);
    } else {
      const double inv = 1.0 / ray.d[a];
      const double t1 = (blo[a] - ray.o[a]) * inv;
      const double t2 = (bhi[a] - ray.o[a]) * inv;
      tn = fmax(tn, fmin(t1, t2));
      tf = fmin(tf, fmax(t1, t2));
    }
  }
  miss |= tn >= tf;
  ray.t_near = tn;
  ray.K = 0;
  if (!miss) {
    const double q = floor((tf - tn) / r.step);
    ray.K = (int)fmin(q, (double)r.max_samples);
  }
  return ray;
}

__device__ __forceinline__ Ray make_ray(const DevModel& m, const RenderArgs& r, int i, int j) {
  return make_ray_box(m.box_lo, m.box_hi, r, i, j);
}

__device__ __forceinline__ void sample_point(const Ray& ray, double step, int k, double (&x)[3]) {
#pragma clang fp contract(off)
  const double t = ray.t_near + ((double)k + 0.5) * step;
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = ray.o[a] + t * ray.d[a];
}

// Partial render: entry parameter t_in of the ray into the region's world
// box (FP64 slab test, the same formula as the model box's) and the range
// [k_lo, k_hi) of samples that can lie in it, widened by one sample on each
// side (the block-owner rule decides the samples at the faces exactly).
__device__ __forceinline__ void region_range(const RenderArgs& r, const Ray& ray, int& k_lo,
                                             int& k_hi, double& t_in) {
#pragma clang fp contract(off)
  double tn = 0.0, tf = __builtin_inf();
  bool miss = ray.K == 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (ray.d[a] == 0.0) {
      miss |= (ray.o[a] < r.reg_box_lo[a]) || (ray.o[a] > r.reg_box_hi[a]);
    } else {
      const double inv = 1.0 / ray.d[a];
      const double t1 = (r.reg_box_lo[a] - ray.o[a]) * inv;
      const double t2 = (r.reg_box_hi[a] - ray.o[a]) * inv;
      tn = fmax(tn, fmin(t1, t2));
      tf = fmin(tf, fmax(t1, t2));
    }
  }
  miss |= tn >= tf;
  if (miss) {
    t_in = __builtin_inf();
    k_lo = k_hi = 0;
    return;
  }
  t_in = tn;
  const double a0 = (tn - ray.t_near) * r.inv_step - 0.5;
  const double a1 = (tf - ray.t_near) * r.inv_step - 0.5;
  k_lo = (int)fmax(floor(a0) - 1.0, 0.0);
  k_hi = (int)fmin(ceil(a1) + 2.0, (double)ray.K);
  if (k_lo > k_hi) k_lo = k_hi;
}

// Knot at the start of span jb of axis a, in FP32: the parameter of a cell
// face for the leap estimates; jb / nsp for uniform knots, else from the
// span records (1 past the last span: the end knot 1).
template <bool GT>
__device__ __forceinline__ float face_knot(const DevModel& m, const SpanRec* __restrict__ R,
                                           const DevBlock* __restrict__ B, int block, int a,
                                           int jb) {
  if (!GT || m.gtab == nullptr || m.gmeta[6 * block + a] < 0)
    return __fdividef((float)jb, (float)B->nsp[a]);
  return jb < B->nsp[a] ? (float)R[B->rec_off[a] + jb].t : 1.f;
}

// Transfer-function coordinate s in [0, 255] of a value (shared by the
// lookup and by the transparency test so both round identically).
__device__ __forceinline__ float tf_coord(float f, float vmin, float inv_range) {
  const float s = (f - vmin) * inv_range;
  return fminf(fmaxf(s, 0.f), 1.f) * 255.f;
}

__device__ __forceinline__ int tf_entry(float s) { return min((int)floorf(s), 254); }

// Transfer function into LDS plus zpre[i] = number of entries below i with
// non-zero opacity (for the transparency test).  All threads take part.
__device__ __forceinline__ void stage_tf(const float* __restrict__ tfp, float4* tf, int* zpre,
                                         int* wtot) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const float4 te = reinterpret_cast<const float4*>(tfp)[tid];
  tf[tid] = te;
  const unsigned long long nzm = __ballot(te.w != 0.f);
  if (lane == 0) wtot[wave] = __popcll(nzm);
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += wtot[w];
  zpre[tid] = base + __popcll(nzm & ((1ull << lane) - 1ull));
  if (tid == kBlock - 1) zpre[256] = base + __popcll(nzm);
  __syncthreads();
}

// True when the transfer function has zero opacity over the whole value
// range of a cell's bounds (FP16 pair lo | hi << 16): every sample in the
// cell then has alpha = 0 exactly.  Two table entries bracket a value, so the
// entries from that of lo to the one after that of hi must all be zero.
__device__ __forceinline__ bool transparent(uint32_t bh, const RenderArgs& r, const int* zpre) {
  const float blo = __half2float(__ushort_as_half((unsigned short)(bh & 0xFFFFu)));
  const float bhi = __half2float(__ushort_as_half((unsigned short)(bh >> 16)));
  return zpre[tf_entry(tf_coord(bhi, r.vmin, r.inv_range)) + 2] ==
         zpre[tf_entry(tf_coord(blo, r.vmin, r.inv_range))];
}

// Transfer function, headlight Phong and one front-to-back "over" step of a
// sample with value and world gradient e (f, df/dx, df/dy, df/dz); returns
// the sample's opacity.
// The colour terms (c_rgb * shade + ks) and the opacity of one sample, which
// do not depend on what lies in front of it.
// diff^m by binary exponentiation (squarings, the set bits of m folded in
// from the lowest); m = 16, the workloads' exponent, is four squarings
// with the same roundings.
__device__ __forceinline__ float spec_pow(float d, int m) {
  if (m == 16) {
    const float d2 = d * d, d4 = d2 * d2, d8 = d4 * d4;
    return d8 * d8;
  }
  float spec = 1.f, bse = d;
  for (int ex = m; ex; ex >>= 1) {
    if (ex & 1) spec *= bse;
    bse *= bse;
  }
  return spec;
}

__device__ __forceinline__ float4 shade_sample(const float4 e, const float (&L)[3], const float4* tf,
                                               const RenderArgs& r) {
  const float s = tf_coord(e.x, r.vmin, r.inv_range);
  const int i0 = tf_entry(s);
  const float w = s - (float)i0;
  const float4 c0 = tf[i0], c1 = tf[i0 + 1];
  const float cr = fmaf(w, c1.x - c0.x, c0.x);
  const float cg = fmaf(w, c1.y - c0.y, c0.y);
  const float cb = fmaf(w, c1.z - c0.z, c0.z);
  const float alpha = fmaf(w, c1.w - c0.w, c0.w);
  // headlight Phong, two-sided; 1 / max(|g|, g0) as one hardware
  // reciprocal square root of max(|g|^2, g0^2)
  const float gg = e.y * e.y + e.z * e.z + e.w * e.w;
  const float inv = __builtin_amdgcn_rsqf(fmaxf(gg, r.g0 * r.g0));
  const float diff = fabsf((e.y * L[0] + e.z * L[1] + e.w * L[2]) * inv);
  const float shade = fmaf(r.kd, diff, r.ka);
  const float ks = r.ks * spec_pow(diff, r.shininess);
  return make_float4(fmaf(cr, shade, ks), fmaf(cg, shade, ks), fmaf(cb, shade, ks), alpha);
}

// front-to-back over of a shaded sample; the opacity update rounds each
// operation
__device__ __forceinline__ void over(const float4 q, float& C0, float& C1, float& C2, float& A) {
  const float om = __fsub_rn(1.f, A);
  const float ta = __fmul_rn(om, q.w);
  C0 = fmaf(ta, q.x, C0);
  C1 = fmaf(ta, q.y, C1);
  C2 = fmaf(ta, q.z, C2);
  A = __fadd_rn(A, ta);
}

__device__ __forceinline__ float shade_over(const float4 e, const float (&L)[3], const float4* tf,
                                            const RenderArgs& r, float& C0, float& C1, float& C2,
                                            float& A) {
  const float4 q = shade_sample(e, L, tf, r);
  over(q, C0, C1, C2, A);
  return q.w;
}

// Transparent stretch in front of a ray's first visible super cell, lane by
// lane: returns the first sample the per-sample loop has to look at (K if
// none).  A sample in a transparent coarse super cell (else in a
// transparent fine one) leaps to the estimated last sample inside that cell
// (FP32 exit through the cell faces at their stored knots, less one step),
// which is then located by the exact rules.  If the landing sample
// lies in the same cell, so does every sample between: the span index per
// axis is monotone along the ray (each rounding step of the position and of
// the parameter map is monotone), so the cell coordinates of a sample in
// between lie between those of the two ends.  All of them then have
// alpha = 0.  If the landing sample lies elsewhere, the leap is undone and
// that cell is crossed sample by sample.  The search stops at the first
// sample whose fine super cell is not transparent; compositing from there
// gives the same pixel as compositing from sample 0.
template <int P, bool MULTI, bool GT = false>
__device__ __forceinline__ int first_visible(const DevModel& m, const RenderArgs& r,
                                             const SpanRec* __restrict__ R, const Ray& ray,
                                             const int* zpre, int k_lo, int k_hi,
                                             const double* __restrict__ EDG) {
  int k = k_lo, from = -1, lvl = 0, cell = -1, noleap = -1, last_c0 = -1;
  bool c0_empty = false;
  while (k < k_hi) {
    double x[3];
    sample_point(ray, r.step, k, x);
    const Loc Lc = locate<P, MULTI, GT>(m, R, x, EDG);
    const DevBlock* __restrict__ B = MULTI ? m.blocks + Lc.block : &m.b0;
    int c[2];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int sh = m.sc_shift[l];
      c[l] = B->sc_off[l] + (((Lc.j[0] >> sh) * B->sc[l][1] + (Lc.j[1] >> sh)) * B->sc[l][2] +
                             (Lc.j[2] >> sh));
    }
    if (from >= 0) {                       // landing sample of a leap at level lvl
      if (c[lvl] != cell) {
        noleap = 2 * cell + lvl;           // no second leap in this cell
        k = from + 1;
      } else {
        ++k;
      }
      from = -1;
      continue;
    }
    if (c[0] != last_c0) {
      c0_empty = transparent(m.scb[0][c[0]], r, zpre);
      last_c0 = c[0];
    }
    lvl = 0;
    if (!c0_empty) {
      if (!transparent(m.scb[1][c[1]], r, zpre)) return k;
      lvl = 1;
    }
    cell = c[lvl];
    int kl = k;
    if (2 * cell + lvl != noleap) {
      const int sh = m.sc_shift[lvl];
      float te = __builtin_inff();
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (ray.d[a] == 0.0) continue;
        const int cc = Lc.j[a] >> sh;
        const int jb = ray.d[a] > 0.0 ? min((cc + 1) << sh, B->nsp[a]) : (cc << sh);
        const float xb = fmaf(face_knot<GT>(m, R, B, Lc.block, a, jb), (float)B->ext[a], (float)B->lo[a]);
        te = fminf(te, (xb - (float)ray.o[a]) * __builtin_amdgcn_rcpf((float)ray.d[a]));
      }
      kl = (int)fminf(floorf(fmaf(te - (float)ray.t_near, (float)r.inv_step, -1.f)),
                      (float)(k_hi - 1));
    }
    if (kl > k + 1) {
      from = k;
      k = kl;
    } else {
      ++k;
    }
  }
  return k_hi;
}

// One 16x16 pixel tile of a frame: one ray per thread.  R, MT: span records
// and basis tables (global pool or an LDS copy); tf, zpre staged in LDS.
// EDG: the block edges (m.edges or an LDS copy).
template <int P, Storage S, bool MULTI, bool PARTIAL = false, bool GT = false>
__device__ __forceinline__ void render_tile(const DevModel& m, const RenderArgs& r, int tile,
                                            const SpanRec* __restrict__ R,
                                            const float* __restrict__ MT, const float4* tf,
                                            const int* zpre, const double* __restrict__ EDG) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int tx = (r.w + kTile - 1) / kTile;
  const int i = (tile % tx) * kTile + (wave & 1) * 8 + (lane & 7);
  const int j = (tile / tx) * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool pix = i < r.w && j < r.h;
  Ray ray;
  ray.K = 0;
  if (pix) ray = make_ray(m, r, i, j);
  float L[3] = {0.f, 0.f, 0.f};
  if (pix) {
    const double dn = sqrt(ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) L[a] = (float)(-ray.d[a] / dn);
  }
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const int64_t pid = (int64_t)j * r.w + i;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
  int k_lo = 0, k_hi = ray.K;
  double t_in = __builtin_inf();
  if constexpr (PARTIAL) {
    if (pix) region_range(r, ray, k_lo, k_hi, t_in);
  }
  const int k0 = pix ? first_visible<P, MULTI, GT>(m, r, R, ray, zpre, k_lo, k_hi, EDG) : 0;
  if (r.alpha)
    for (int q = 0; q < k0; ++q) r.alpha[pid * r.alpha_stride + q] = 0.f;
  int used = k0, nev = 0;
  bool done = false;
  int last_mc = -1;
  bool last_empty = false;
  for (int k = k0;; ++k) {
    const bool act = pix && !done && k < k_hi;
    if (__ballot(act) == 0) break;                 // whole wave finished
    if (!act) continue;
    double x[3];
    sample_point(ray, r.step, k, x);
    // Skip the evaluation where the transfer function is zero over the
    // value bounds of the macro cell: such a sample has alpha = 0 exactly
    // and leaves C and A unchanged.  The verdict is kept while the ray
    // stays in the same cell.  The bounds of the cell of the guessed spans
    // are fetched while the guesses are checked (reloaded in the rare case
    // that the exact spans lie in another cell).
    Probe q;
    int mcg;
    uint32_t bh = 0;
    Loc Lc;
    auto locate_in = [&](const DevBlock* B, const double (&xc)[3]) {
      probe_spans<GT>(m, R, xc, B, q);
      mcg = macro_cell(m, q.B, q.j);
      if (mcg != last_mc) bh = m.mcb[mcg];
      Lc = finish(m, R, q);
    };
    if constexpr (MULTI) {
      // Most waves have all their samples of this step in one block: then
      // its record is read once for the wave, through the scalar cache,
      // instead of by every lane.
      double xc[3];
      probe_owner(m, x, EDG, q, xc);
      const int bu = __builtin_amdgcn_readfirstlane(q.block);
      if (__builtin_amdgcn_ballot_w64(q.block != bu) == 0)
        locate_in(m.blocks + bu, xc);
      else
        locate_in(m.blocks + q.block, xc);
    } else {
      q = probe<MULTI, GT>(m, R, x, EDG);
      mcg = macro_cell(m, q.B, q.j);
      if (mcg != last_mc) bh = m.mcb[mcg];
      Lc = finish(m, R, q);
    }
    if (Lc.mc != last_mc) {
      if (Lc.mc != mcg) bh = m.mcb[Lc.mc];
      last_empty = transparent(bh, r, zpre);
      last_mc = Lc.mc;
    }
    // a partial render skips the samples owned by blocks outside its region
    bool outside = false;
    if constexpr (PARTIAL) {
#pragma unroll
      for (int a = 0; a < 3; ++a) outside |= q.b[a] < r.reg_lo[a] || q.b[a] >= r.reg_hi[a];
    }
    const bool empty = last_empty || outside;
    float alpha = 0.f;
    if (!empty) {
      const float4 e = evaluate<P, S, !MULTI>(Lc, rs, MT, m.mat_stride, m.imat);
      ++nev;
      alpha = shade_over(e, L, tf, r, C0, C1, C2, A);
    }
    used = k + 1;
    if (r.alpha) r.alpha[pid * r.alpha_stride + k] = alpha;
    done = A >= r.ert_alpha;
  }
  if (pix) {
    if (r.key)    // entry key: of the region, else of the model box
      r.key[pid] = PARTIAL ? t_in : (ray.K > 0 ? ray.t_near : __builtin_inf());
    reinterpret_cast<float4*>(r.rgba)[pid] = make_float4(C0, C1, C2, A);
    if (r.nsamp) reinterpret_cast<int2*>(r.nsamp)[pid] = make_int2(ray.K, used);
    if (r.neval) r.neval[pid] = nev;
  }
}

// Broadcast of lane t of each group of four lanes (a DPP quad permute).
template <int T>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), T * 0x55, 0xF, 0xF, false));
}

template <int T>
__device__ __forceinline__ float4 quad_bcast4(float4 v) {
  return make_float4(quad_bcast<T>(v.x), quad_bcast<T>(v.y), quad_bcast<T>(v.z), quad_bcast<T>(v.w));
}

// One 8x8 pixel tile of a frame with four lanes per ray (16 rays per wave):
// lane s of a ray's group evaluates samples k0 + s, k0 + s + 4, ...; the
// group then composites its four samples in ray order, every lane of the
// group carrying the same C and A, with the same operations as one lane
// stepping through them, and stops at the same sample (early ray
// termination, the end of the ray).  A long ray takes a quarter of the
// lockstep iterations, which shortens the drain at the end of a frame.
template <int P, Storage S, bool MULTI, bool GT = false>
__device__ __forceinline__ void render_tile4(const DevModel& m, const RenderArgs& r, int tile,
                                             const SpanRec* __restrict__ R,
                                             const float* __restrict__ MT, const float4* tf,
                                             const int* zpre) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, s = lane & 3;
  const int tx = (r.w + 7) / 8;
  const int i = (tile % tx) * 8 + (wave & 1) * 4 + ((lane >> 2) & 3);
  const int j = (tile / tx) * 8 + (wave >> 1) * 4 + (lane >> 4);
  const bool pix = i < r.w && j < r.h;
  Ray ray;
  ray.K = 0;
  if (pix) ray = make_ray(m, r, i, j);
  // the ray's headlight direction, kept in LDS (read once per evaluated
  // sample) rather than in three registers for the whole loop
  __shared__ float4 lray[kBlock / 4];
  if (pix && s == 0) {
    const double dn = sqrt(ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
    lray[threadIdx.x >> 2] = make_float4((float)(-ray.d[0] / dn), (float)(-ray.d[1] / dn),
                                         (float)(-ray.d[2] / dn), 0.f);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const int pid = j * r.w + i;                     // w, h <= 16384
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
  const int k_hi = ray.K;
  // The four lanes of a ray search a quarter of it each for the first
  // sample in a non-transparent fine super cell (the quarter's end if
  // none): the first of the four results is that of the whole ray, and the
  // quarters at the ray's end with no such sample are left out of the loop
  // (k_end), their samples all having alpha = 0.
  const int seg = (k_hi + 3) >> 2;
  int kv = k_hi, emp = 1;
  if (pix) {
    const int lo = min(k_hi, s * seg), hi = min(k_hi, lo + seg);
    const int f = first_visible<P, MULTI, GT>(m, r, R, ray, zpre, lo, hi, m.edges);
    kv = f < hi ? f : k_hi;
    emp = f < hi ? 0 : 1;
  }
  const int k0 = min(min(__float_as_int(quad_bcast<0>(__int_as_float(kv))),
                         __float_as_int(quad_bcast<1>(__int_as_float(kv)))),
                     min(__float_as_int(quad_bcast<2>(__int_as_float(kv))),
                         __float_as_int(quad_bcast<3>(__int_as_float(kv)))));
  const int e = (__float_as_int(quad_bcast<0>(__int_as_float(emp)))) |
                (__float_as_int(quad_bcast<1>(__int_as_float(emp))) << 1) |
                (__float_as_int(quad_bcast<2>(__int_as_float(emp))) << 2) |
                (__float_as_int(quad_bcast<3>(__int_as_float(emp))) << 3);
  // first quarter from which every later one is empty (4: none)
  const int qe = (e & 8) ? ((e & 4) ? ((e & 2) ? ((e & 1) ? 0 : 1) : 2) : 3) : 4;
  const int k_end = min(k_hi, qe * seg);
  if (r.alpha && pix)
    for (int q = s; q < k0; q += 4) r.alpha[(int64_t)pid * r.alpha_stride + q] = 0.f;
  int used = k0, nev = 0;
  bool done = false;
  int last_mc = -1;
  bool last_empty = false;
  for (int kb = k0;; kb += 4) {
    const bool act = pix && !done && kb < k_end;     // the same in the four lanes of a ray
    if (__ballot(act) == 0) break;
    if (!act) continue;
    const int k = kb + s;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    bool ev = false;
    if (k < k_end) {
      double x[3];
      sample_point(ray, r.step, k, x);
      Probe pr = probe<MULTI, GT>(m, R, x);
      const int mcg = macro_cell(m, pr.B, pr.j);
      uint32_t bh = 0;
      if (mcg != last_mc) bh = m.mcb[mcg];
      const Loc Lc = finish(m, R, pr);
      if (Lc.mc != last_mc) {
        if (Lc.mc != mcg) bh = m.mcb[Lc.mc];
        last_empty = transparent(bh, r, zpre);
        last_mc = Lc.mc;
      }
      if (!last_empty) {
        const float4 e = evaluate<P, S, !MULTI>(Lc, rs, MT, m.mat_stride, m.imat);
        const float4 l4 = lray[threadIdx.x >> 2];   // written by lane 0 of the ray, same wave
        const float L[3] = {l4.x, l4.y, l4.z};
        q = shade_sample(e, L, tf, r);
        ev = true;
      }
    }
    // The group's four samples in ray order.  A sample that was not
    // evaluated (transparent cell, past the end of the ray) enters as
    // colour 0 and opacity 0, for which "over" leaves C and A exactly
    // unchanged, so every sample goes through the same steps; after the
    // first sample that reaches the termination opacity the others are
    // masked.  In an iteration where no lane of the wave evaluated, the
    // four steps change nothing and are left out.
    if (__ballot(ev) != 0) {
      const float4 q0 = quad_bcast4<0>(q), q1 = quad_bcast4<1>(q), q2 = quad_bcast4<2>(q),
                   q3 = quad_bcast4<3>(q);
      int stop = 0;                // 1 + index of the terminating sample, 0: none
      auto step = [&](float4 qt, int t) {
        const bool live = stop == 0;
        qt.w = live ? qt.w : 0.f;
        over(qt, C0, C1, C2, A);
        if (live && A >= r.ert_alpha) stop = t + 1;
      };
      step(q0, 0);
      step(q1, 1);
      step(q2, 2);
      step(q3, 3);
      done = stop != 0;
      used = done ? kb + stop : min(kb + 4, k_end);
    } else {
      used = min(kb + 4, k_end);
    }
    nev += (ev && k < used) ? 1 : 0;
    if (r.alpha && k < used) r.alpha[(int64_t)pid * r.alpha_stride + k] = ev ? q.w : 0.f;
  }
  if (pix && !done) {               // the transparent quarters at the end leave C and A as they are
    if (r.alpha)
      for (int q = k_end + s; q < k_hi; q += 4) r.alpha[(int64_t)pid * r.alpha_stride + q] = 0.f;
    used = k_hi;
  }
  // evaluated samples of the ray: the sum over its four lanes
  {
    const int n1 = __float_as_int(quad_bcast<1>(__int_as_float(nev)));
    const int n2 = __float_as_int(quad_bcast<2>(__int_as_float(nev)));
    const int n3 = __float_as_int(quad_bcast<3>(__int_as_float(nev)));
    const int n0 = __float_as_int(quad_bcast<0>(__int_as_float(nev)));
    nev = n0 + n1 + n2 + n3;
  }
  if (pix && s == 0) {
    if (r.key) r.key[pid] = ray.K > 0 ? ray.t_near : __builtin_inf();
    reinterpret_cast<float4*>(r.rgba)[pid] = make_float4(C0, C1, C2, A);
    if (r.nsamp) reinterpret_cast<int2*>(r.nsamp)[pid] = make_int2(ray.K, used);
    if (r.neval) r.neval[pid] = nev;
  }
}

// Tile rows are dealt round-robin to the XCDs (row % 8), so every XCD
// gets rows from the whole frame; workgroups resident on one XCD still
// cover neighbouring rows of its share.
__device__ __forceinline__ int frame_tile(int bid, int tx, int ty) {
  const int i = xcd_tile(bid, tx * ty);
  int base = 0;
  for (int c = 0; c < 8; ++c) {
    const int nr = (ty - c + 7) >> 3;
    if (i < base + nr * tx) {
      const int o = i - base;
      return ((o / tx) * 8 + c) * tx + (o % tx);
    }
    base += nr * tx;
  }
  return 0;
}

// LDSREC: single-block model whose span records and basis tables are copied
// into LDS once per workgroup.
// GM: basis tables read from the global pool (models whose tables exceed
// kMatsLds floats; multi-block kernels only), else from an LDS copy.
// EL: multi-block model whose block edges (at most kEdgesLds values) are
// copied into LDS, so that each sample's owner check reads them there.
constexpr int kEdgesLds = 256;

template <int P, Storage S, bool MULTI, bool LDSREC, bool PARTIAL = false, bool GT = false,
          bool QUAD = false, bool GM = false, bool EL = false>
__global__ __launch_bounds__(kBlock) void render_k(DevModel m, RenderArgs r) {
  extern __shared__ float4 dyn[];
  __shared__ float4 lmats[LDSREC || GM ? 1 : kMatsLds / 4];
  __shared__ float4 tf[256];
  __shared__ int zpre[257];
  __shared__ int wtot[kBlock / kWave];
  __shared__ double ledges[EL ? kEdgesLds : 1];
  const double* EDG = m.edges;
  if constexpr (EL) {
    for (int q = threadIdx.x; q < m.n_edges; q += kBlock) ledges[q] = m.edges[q];
    EDG = ledges;                  // read after stage_tf's barriers
  }
  const SpanRec* R = m.rec;
  const float* MT = m.mats;
  if constexpr (LDSREC) {
    SpanRec* lr = reinterpret_cast<SpanRec*>(dyn);
    float* lm = reinterpret_cast<float*>(lr + m.n_rec);
    for (int q = threadIdx.x; q < m.n_rec * 2; q += kBlock)
      reinterpret_cast<float4*>(lr)[q] = reinterpret_cast<const float4*>(m.rec)[q];
    for (int q = threadIdx.x; q < m.n_mats * m.mat_stride / 4; q += kBlock)
      reinterpret_cast<float4*>(lm)[q] = reinterpret_cast<const float4*>(m.mats)[q];
    R = lr;
    MT = lm;
  } else if constexpr (!GM) {
    for (int q = threadIdx.x; q < m.n_mats * m.mat_stride / 4; q += kBlock)
      lmats[q] = reinterpret_cast<const float4*>(m.mats)[q];
    MT = reinterpret_cast<const float*>(lmats);
  }
  stage_tf(r.tf, tf, zpre, wtot);
  if constexpr (QUAD) {
    static_assert(!PARTIAL, "four lanes per ray: full frames");
    const int tx = (r.w + 7) / 8, ty = (r.h + 7) / 8;
    render_tile4<P, S, MULTI, GT>(m, r, frame_tile(blockIdx.x, tx, ty), R, MT, tf, zpre);
  } else {
    const int tx = (r.w + kTile - 1) / kTile, ty = (r.h + kTile - 1) / kTile;
    render_tile<P, S, MULTI, PARTIAL, GT>(m, r, frame_tile(blockIdx.x, tx, ty), R, MT, tf, zpre, EDG);
  }
}

// ------------------------------------------------------------------ K8: isosurface
// First-hit isosurface on the volume renderer's ray schedule: a sample is on
// side 1 when f >= iso; the surface lies between the first two consecutive
// samples whose sides differ, at the linear interpolation of f between
// them; the hit is shaded with the volume renderer's headlight Phong
// (surface colour iso_rgb, opacity 1).  The value bounds of a macro cell
// (its control points' range, widened beyond the FP32 evaluation error and
// rounded outwards to FP16) contain every evaluation in the cell, so a cell
// whose lower bound is >= iso puts all its samples on side 1, one whose
// upper bound is < iso on side 0: the sides an evaluation would give.  The
// value of such a sample is evaluated only if it brackets the hit.  The
// same test on the coarse and fine super cells lets a ray leap across a
// super cell wholly on one side.
__device__ __forceinline__ int iso_side(uint32_t bh, float iso) {
  const float blo = __half2float(__ushort_as_half((unsigned short)(bh & 0xFFFFu)));
  const float bhi = __half2float(__ushort_as_half((unsigned short)(bh >> 16)));
  return iso <= blo ? 1 : (iso > bhi ? 0 : -1);
}

template <int P, Storage S, bool MULTI, bool GT = false>
__device__ __forceinline__ void iso_tile(const DevModel& m, const RenderArgs& r, int tile,
                                         const SpanRec* __restrict__ R,
                                         const float* __restrict__ MT) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int tx = (r.w + kTile - 1) / kTile;
  const int i = (tile % tx) * kTile + (wave & 1) * 8 + (lane & 7);
  const int j = (tile / tx) * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool pix = i < r.w && j < r.h;
  Ray ray;
  ray.K = 0;
  if (pix) ray = make_ray(m, r, i, j);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const int64_t pid = (int64_t)j * r.w + i;
  int hit = -1, nev = 0, side_prev = -1;
  float fprev = 0.f, fa = 0.f, fb = 0.f;
  bool known = false;                    // fprev holds the value of sample k - 1
  bool back = false;                     // this step evaluates sample k - 1 (hit found at k)
  // cached sides of the last coarse, fine and macro cell (-1: undecided)
  int last_c[3] = {-1, -1, -1}, side_c[3] = {-1, -1, -1};
  // leap state: origin sample, level and cell of a pending leap; the cell
  // (2 * cell + level) where a leap failed and is not tried again
  int k = 0, from = -1, lvl = 0, cell = -1, noleap = -1;
  // One located sample and at most one value query per lane and step, so
  // that the lanes needing a value share one evaluation.
  for (;;) {
    const bool act = pix && hit < 0 && k < ray.K;
    if (__ballot(act) == 0) break;       // whole wave finished
    if (!act) continue;
    double x[3];
    sample_point(ray, r.step, back ? k - 1 : k, x);
    const Loc Lc = locate<P, MULTI, GT>(m, R, x);
    const DevBlock* __restrict__ B = MULTI ? m.blocks + Lc.block : &m.b0;
    int c[3];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int sh = m.sc_shift[l];
      c[l] = B->sc_off[l] + (((Lc.j[0] >> sh) * B->sc[l][1] + (Lc.j[1] >> sh)) * B->sc[l][2] +
                             (Lc.j[2] >> sh));
    }
    c[2] = Lc.mc;
    int lv = 3;
    if (!back && from < 0) {
      uint32_t bh[3];
#pragma unroll
      for (int l = 0; l < 3; ++l)
        if (c[l] != last_c[l]) bh[l] = l < 2 ? m.scb[l][c[l]] : m.mcb[c[l]];
#pragma unroll
      for (int l = 0; l < 3; ++l)
        if (c[l] != last_c[l]) {
          side_c[l] = iso_side(bh[l], r.iso);
          last_c[l] = c[l];
        }
      lv = side_c[0] >= 0 ? 0 : (side_c[1] >= 0 ? 1 : (side_c[2] >= 0 ? 2 : 3));
    }
    const int sdec = lv < 3 ? side_c[lv] : -1;
    const bool need = back || (from < 0 && (sdec < 0 || (k > 0 && sdec != side_prev)));
    float f = 0.f;
    if (need) {
      f = evaluate<P, S, !MULTI>(Lc, rs, MT, m.mat_stride, m.imat).x;
      ++nev;
    }
    if (back) {                          // the value before the hit
      fa = f;
      hit = k;
      continue;
    }
    if (from >= 0) {                     // landing sample of a leap at level lvl
      if (c[lvl] != cell) {              // left the cell: undo, step from the origin
        noleap = 2 * cell + lvl;
        k = from + 1;
      } else {                           // every sample up to here had the origin's side
        known = false;
        ++k;
      }
      from = -1;
      continue;
    }
    const int side = sdec >= 0 ? sdec : (f >= r.iso ? 1 : 0);
    if (k > 0 && side != side_prev) {
      fb = f;
      if (known) {
        fa = fprev;
        hit = k;
      } else {
        back = true;
      }
      continue;
    }
    side_prev = side;
    fprev = f;
    known = need;
    // A super cell on one side of the level: leap to the estimated last
    // sample inside it (FP32 exit through the cell faces at their stored
    // knots, less one step), located next by the exact rules.  If that
    // sample lies in the same cell, so does every sample between (the span
    // index per axis is monotone along the ray), which all have this side;
    // otherwise the leap is undone.
    int kl = k;
    if (lv < 2 && 2 * c[lv] + lv != noleap) {
      const int sh = m.sc_shift[lv];
      float te = __builtin_inff();
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (ray.d[a] == 0.0) continue;
        const int cc = Lc.j[a] >> sh;
        const int jb = ray.d[a] > 0.0 ? min((cc + 1) << sh, B->nsp[a]) : (cc << sh);
        const float xb = fmaf(face_knot<GT>(m, R, B, Lc.block, a, jb), (float)B->ext[a], (float)B->lo[a]);
        te = fminf(te, (xb - (float)ray.o[a]) * __builtin_amdgcn_rcpf((float)ray.d[a]));
      }
      kl = (int)fminf(floorf(fmaf(te - (float)ray.t_near, (float)r.inv_step, -1.f)),
                      (float)(ray.K - 1));
    }
    if (kl > k + 1) {
      from = k;
      lvl = lv;
      cell = c[lv];
      k = kl;
    } else {
      ++k;
    }
  }
  float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
  double depth = __builtin_inf();
  if (pix && hit > 0) {
    // fa and fb lie on different sides of iso, so w is in [0, 1]
    const float w = (r.iso - fa) / (fb - fa);
    double xs[3];
    {
#pragma clang fp contract(off)
      depth = ray.t_near + (((double)(hit - 1) + 0.5) + (double)w) * r.step;
#pragma unroll
      for (int a = 0; a < 3; ++a) xs[a] = ray.o[a] + depth * ray.d[a];
    }
    const Loc Ls = locate<P, MULTI, GT>(m, R, xs);
    const float4 e = evaluate<P, S, !MULTI>(Ls, rs, MT, m.mat_stride, m.imat);
    ++nev;
    const double dn = sqrt(ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
    float L[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) L[a] = (float)(-ray.d[a] / dn);
    const float gg = e.y * e.y + e.z * e.z + e.w * e.w;
    const float inv = __builtin_amdgcn_rsqf(fmaxf(gg, r.g0 * r.g0));
    const float diff = fabsf((e.y * L[0] + e.z * L[1] + e.w * L[2]) * inv);
    const float shade = fmaf(r.kd, diff, r.ka);
    const float ks = r.ks * spec_pow(diff, r.shininess);
    out = make_float4(fmaf(r.iso_rgb[0], shade, ks), fmaf(r.iso_rgb[1], shade, ks),
                      fmaf(r.iso_rgb[2], shade, ks), 1.f);
  }
  if (pix) {
    reinterpret_cast<float4*>(r.rgba)[pid] = out;
    if (r.key) r.key[pid] = depth;
    if (r.nsamp) reinterpret_cast<int2*>(r.nsamp)[pid] = make_int2(ray.K, hit);
    if (r.neval) r.neval[pid] = nev;
  }
}

// Four lanes per ray (single-block full frames): lane s of a ray's group
// decides the side of samples s, s + 4, ... (by the bounds of the first
// cell level that decides it, else by its value), and the group takes the
// first side change in ray order.  A group whose last sample lies in a
// super cell wholly on one side leaps, as the one-lane search does, to the
// estimated last sample inside that cell; the leap holds if the group's
// next first sample lies in the same cell (every sample between then does:
// the span index per axis is monotone along the ray) and is undone
// otherwise.  Two lanes then evaluate the samples around the hit, and the
// hit point is shaded as in the one-lane search.
template <int P, Storage S, bool MULTI, bool GT = false>
__device__ __forceinline__ void iso_tile4(const DevModel& m, const RenderArgs& r, int tile,
                                          const SpanRec* __restrict__ R,
                                          const float* __restrict__ MT) {
  static_assert(!MULTI, "four lanes per ray: single-block models");
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, s = lane & 3;
  const int tx = (r.w + 7) / 8;
  const int i = (tile % tx) * 8 + (wave & 1) * 4 + ((lane >> 2) & 3);
  const int j = (tile / tx) * 8 + (wave >> 1) * 4 + (lane >> 4);
  const bool pix = i < r.w && j < r.h;
  Ray ray;
  ray.K = 0;
  if (pix) ray = make_ray(m, r, i, j);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
  const int64_t pid = (int64_t)j * r.w + i;
  const DevBlock* __restrict__ B = &m.b0;
  auto bcast = [](int v, int t) {
    const float f = __int_as_float(v);
    return __float_as_int(t == 0 ? quad_bcast<0>(f) : t == 1 ? quad_bcast<1>(f)
                          : t == 2 ? quad_bcast<2>(f) : quad_bcast<3>(f));
  };
  int hit = -1, nev = 0, side_prev = -1;          // side_prev: the side of sample kb - 1
  // cached sides of the last coarse, fine and macro cell (-1: undecided)
  int last_c[3] = {-1, -1, -1}, side_c[3] = {-1, -1, -1};
  // leap state of the group: first skipped sample, level and cell of a
  // pending leap; the cell (2 * cell + level) where a leap failed
  int kb = 0, from = -1, lvl = 0, cell = -1, noleap = -1;
  for (;;) {
    const bool act = pix && hit < 0 && kb < ray.K;   // the same in the four lanes of a ray
    if (__ballot(act) == 0) break;                  // whole wave finished
    if (!act) continue;
    const int k = kb + s;
    int side = -1;                                  // -1: past the end of the ray
    int c[3] = {-1, -1, -1}, lv = 3, js[3] = {0, 0, 0};
    if (k < ray.K) {
      double x[3];
      sample_point(ray, r.step, k, x);
      const Loc Lc = locate<P, MULTI, GT>(m, R, x);
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        const int sh = m.sc_shift[l];
        c[l] = B->sc_off[l] + (((Lc.j[0] >> sh) * B->sc[l][1] + (Lc.j[1] >> sh)) * B->sc[l][2] +
                               (Lc.j[2] >> sh));
      }
      c[2] = Lc.mc;
      uint32_t bh[3];
#pragma unroll
      for (int l = 0; l < 3; ++l)
        if (c[l] != last_c[l]) bh[l] = l < 2 ? m.scb[l][c[l]] : m.mcb[c[l]];
#pragma unroll
      for (int l = 0; l < 3; ++l)
        if (c[l] != last_c[l]) {
          side_c[l] = iso_side(bh[l], r.iso);
          last_c[l] = c[l];
        }
      lv = side_c[0] >= 0 ? 0 : (side_c[1] >= 0 ? 1 : (side_c[2] >= 0 ? 2 : 3));
      if (lv < 3) {
        side = side_c[lv];
      } else {
        side = evaluate<P, S, !MULTI>(Lc, rs, MT, m.mat_stride, m.imat).x >= r.iso ? 1 : 0;
        ++nev;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) js[a] = Lc.j[a];
    }
    if (from >= 0) {                                // landing of a leap at level lvl
      const int cl = bcast(lvl == 0 ? c[0] : c[1], 0);
      if (cl != cell) {                             // left the cell: undo
        noleap = 2 * cell + lvl;
        kb = from;
        from = -1;
        continue;
      }
      from = -1;                                    // the samples passed had side side_prev
    }
    // the first side change among the group's samples, in ray order
    int sp = side_prev, th = -1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int st = bcast(side, t);
      if (th < 0 && st >= 0) {
        if (kb + t > 0 && st != sp) th = t;
        else sp = st;
      }
    }
    if (th >= 0) {
      hit = kb + th;
      continue;
    }
    side_prev = sp;
    // leap from the group's last sample when its super cell (level 0 or 1)
    // lies wholly on one side: to the estimated last sample inside the cell
    // (FP32 exit through the cell faces at their stored knots, less one step)
    int kl = kb + 4;
    const int lv3 = bcast(lv, 3);
    const int c3 = bcast(lv == 0 ? c[0] : c[1], 3);
    if (lv3 < 2 && 2 * c3 + lv3 != noleap) {
      const int sh = m.sc_shift[lv3];
      float te = __builtin_inff();
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ja = bcast(js[a], 3);
        if (ray.d[a] == 0.0) continue;
        const int cc = ja >> sh;
        const int jb = ray.d[a] > 0.0 ? min((cc + 1) << sh, B->nsp[a]) : (cc << sh);
        const float xb = fmaf(face_knot<GT>(m, R, B, 0, a, jb), (float)B->ext[a], (float)B->lo[a]);
        te = fminf(te, (xb - (float)ray.o[a]) * __builtin_amdgcn_rcpf((float)ray.d[a]));
      }
      kl = max(kb + 4, (int)fminf(floorf(fmaf(te - (float)ray.t_near, (float)r.inv_step, -1.f)),
                                  (float)(ray.K - 1)));
    }
    if (kl > kb + 4) {
      from = kb + 4;
      lvl = lv3;
      cell = c3;
    }
    kb = kl;
  }
  // the values at the two samples around the hit (lanes 0 and 1), then the
  // hit point, as in the one-lane search
  float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
  double depth = __builtin_inf();
  if (pix && hit > 0) {
    float f = 0.f;
    if (s < 2) {
      double x[3];
      sample_point(ray, r.step, hit - 1 + s, x);
      const Loc Lc = locate<P, MULTI, GT>(m, R, x);
      f = evaluate<P, S, !MULTI>(Lc, rs, MT, m.mat_stride, m.imat).x;
      ++nev;
    }
    const float fa = quad_bcast<0>(f), fb = quad_bcast<1>(f);
    // fa and fb lie on different sides of iso, so w is in [0, 1]
    const float w = (r.iso - fa) / (fb - fa);
    double xs[3];
    {
#pragma clang fp contract(off)
      depth = ray.t_near + (((double)(hit - 1) + 0.5) + (double)w) * r.step;
#pragma unroll
      for (int a = 0; a < 3; ++a) xs[a] = ray.o[a] + depth * ray.d[a];
    }
    const Loc Ls = locate<P, MULTI, GT>(m, R, xs);
    const float4 e = evaluate<P, S, !MULTI>(Ls, rs, MT, m.mat_stride, m.imat);
    if (s == 0) ++nev;
    const double dn = sqrt(ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
    float L[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) L[a] = (float)(-ray.d[a] / dn);
    const float gg = e.y * e.y + e.z * e.z + e.w * e.w;
    const float inv = __builtin_amdgcn_rsqf(fmaxf(gg, r.g0 * r.g0));
    const float diff = fabsf((e.y * L[0] + e.z * L[1] + e.w * L[2]) * inv);
    const float shade = fmaf(r.kd, diff, r.ka);
    const float ks = r.ks * spec_pow(diff, r.shininess);
    out = make_float4(fmaf(r.iso_rgb[0], shade, ks), fmaf(r.iso_rgb[1], shade, ks),
                      fmaf(r.iso_rgb[2], shade, ks), 1.f);
  }
  // values evaluated for the ray: the sum over its four lanes
  nev = bcast(nev, 0) + bcast(nev, 1) + bcast(nev, 2) + bcast(nev, 3);
  if (pix && s == 0) {
    reinterpret_cast<float4*>(r.rgba)[pid] = out;
    if (r.key) r.key[pid] = depth;
    if (r.nsamp) reinterpret_cast<int2*>(r.nsamp)[pid] = make_int2(ray.K, hit);
    if (r.neval) r.neval[pid] = nev;
  }
}

template <int P, Storage S, bool MULTI, bool LDSREC, bool GT = false, bool QUAD = false>
__global__ __launch_bounds__(kBlock) void iso_k(DevModel m, RenderArgs r) {
  extern __shared__ float4 dyn[];
  const SpanRec* R = m.rec;
  const float* MT = m.mats;
  if constexpr (LDSREC) {
    SpanRec* lr = reinterpret_cast<SpanRec*>(dyn);
    float* lm = reinterpret_cast<float*>(lr + m.n_rec);
    for (int q = threadIdx.x; q < m.n_rec * 2; q += kBlock)
      reinterpret_cast<float4*>(lr)[q] = reinterpret_cast<const float4*>(m.rec)[q];
    for (int q = threadIdx.x; q < m.n_mats * m.mat_stride / 4; q += kBlock)
      reinterpret_cast<float4*>(lm)[q] = reinterpret_cast<const float4*>(m.mats)[q];
    R = lr;
    MT = lm;
    __syncthreads();
  }
  if constexpr (QUAD) {
    const int tx = (r.w + 7) / 8, ty = (r.h + 7) / 8;
    iso_tile4<P, S, MULTI, GT>(m, r, frame_tile(blockIdx.x, tx, ty), R, MT);
  } else {
    const int tx = (r.w + kTile - 1) / kTile, ty = (r.h + kTile - 1) / kTile;
    iso_tile<P, S, MULTI, GT>(m, r, frame_tile(blockIdx.x, tx, ty), R, MT);
  }
}

// ------------------------------------------------------------------ K9: local-filter volumes
// The same ray caster over a volume of samples reconstructed by a local
// filter (the baselines the paper compares MFA queries with), or over the
// analytic Marschner-Lobb field (its quality study's ground truth).  Every
// sample up to the termination is evaluated (no empty-space skipping).
template <int KIND, int K>
__device__ __forceinline__ void filter_weights(float t, float (&w)[K], float (&dw)[K]) {
  if constexpr (KIND == MFA_FILTER_TRILINEAR) {
    w[0] = 1.f - t;
    w[1] = t;
    dw[0] = -1.f;
    dw[1] = 1.f;
  } else if constexpr (KIND == MFA_FILTER_CATMULL_ROM) {
    const float t2 = t * t, t3 = t2 * t;
    w[0] = 0.5f * (-t3 + 2.f * t2 - t);
    w[1] = 0.5f * (3.f * t3 - 5.f * t2 + 2.f);
    w[2] = 0.5f * (-3.f * t3 + 4.f * t2 + t);
    w[3] = 0.5f * (t3 - t2);
    dw[0] = 0.5f * (-3.f * t2 + 4.f * t - 1.f);
    dw[1] = 0.5f * (9.f * t2 - 10.f * t);
    dw[2] = 0.5f * (-9.f * t2 + 8.f * t + 1.f);
    dw[3] = 0.5f * (3.f * t2 - 2.f * t);
  } else {
    const float t2 = t * t, t3 = t2 * t, s = 1.f - t;
    constexpr float sixth = 1.f / 6.f;
    w[0] = s * s * s * sixth;
    w[1] = (3.f * t3 - 6.f * t2 + 4.f) * sixth;
    w[2] = (-3.f * t3 + 3.f * t2 + 3.f * t + 1.f) * sixth;
    w[3] = t3 * sixth;
    dw[0] = -0.5f * s * s;
    dw[1] = (9.f * t2 - 12.f * t) * sixth;
    dw[2] = (-9.f * t2 + 6.f * t + 3.f) * sixth;
    dw[3] = 0.5f * t2;
  }
}

template <int KIND>
__device__ __forceinline__ float4 volume_field(const VolArgs& v, const double (&x)[3]) {
  if constexpr (KIND == MFA_FIELD_MARSCHNER_LOBB) {
    constexpr float kPi = 3.14159265358979f, kFm = 6.f, kAlpha = 0.25f;
    constexpr float kDen = 2.f * (1.f + kAlpha);
    const float X = (float)x[0], Y = (float)x[1], Z = (float)x[2];
    const float rr = sqrtf(X * X + Y * Y);
    const float inner = 2.f * kPi * kFm * cosf(0.5f * kPi * rr);
    const float f = (1.f - sinf(0.5f * kPi * Z) + kAlpha * (1.f + cosf(inner))) / kDen;
    const float drho = sinf(inner) * (2.f * kPi * kFm) * sinf(0.5f * kPi * rr) * (0.5f * kPi);
    const float q = rr > 0.f ? kAlpha * drho / (rr * kDen) : 0.f;
    return make_float4(f, q * X, q * Y, -0.5f * kPi * cosf(0.5f * kPi * Z) / kDen);
  } else {
    constexpr int K = KIND == MFA_FILTER_TRILINEAR ? 2 : 4;
    constexpr int OFF = KIND == MFA_FILTER_TRILINEAR ? 0 : -1;
    int c[3];
    float w[3][K], dw[3][K];
    // grid coordinate in FP64 through the host's 1 / h (a cell face may go
    // to either neighbour, between which every filter here is continuous)
    bool inner = v.bytes < 0xFFFFFFF0ll;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double g = clampd((x[a] - v.lo[a]) * v.inv_hd[a], 0.0, (double)(v.n[a] - 1));
      c[a] = min((int)floor(g), v.n[a] - 2);
      filter_weights<KIND, K>((float)(g - (double)c[a]), w[a], dw[a]);
      inner = inner && c[a] + OFF >= 0 && c[a] + OFF + K - 1 <= v.n[a] - 1;
    }
    float f = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    auto contract = [&](auto&& row) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        float y = 0.f, yy = 0.f, yz = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float sv[K];
          row(i, j, sv);
          float z = 0.f, zd = 0.f;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            z = fmaf(w[2][k], sv[k], z);
            zd = fmaf(dw[2][k], sv[k], zd);
          }
          y = fmaf(w[1][j], z, y);
          yy = fmaf(dw[1][j], z, yy);
          yz = fmaf(w[1][j], zd, yz);
        }
        f = fmaf(w[0][i], y, f);
        fx = fmaf(dw[0][i], y, fx);
        fy = fmaf(w[0][i], yy, fy);
        fz = fmaf(w[0][i], yz, fz);
      }
    };
    if (inner) {
      // the whole stencil inside the grid: rows of K consecutive samples,
      // one vector load each at a lane offset plus a uniform row offset
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(v.v, v.bytes);
      const uint32_t n1 = (uint32_t)v.n[1], n2 = (uint32_t)v.n[2];
      const uint32_t e0 = ((uint32_t)(c[0] + OFF) * n1 + (uint32_t)(c[1] + OFF)) * n2 + (uint32_t)(c[2] + OFF);
      contract([&](int i, int j, float (&sv)[K]) {
        uint32_t wd[K];
        load_words<K>(rs, e0 * 4u, ((uint32_t)i * n1 * n2 + (uint32_t)j * n2) * 4u, wd);
#pragma unroll
        for (int k = 0; k < K; ++k) sv[k] = __uint_as_float(wd[k]);
      });
    } else {
      // stencil indices outside the grid repeat the edge sample
      int idx[3][K];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < K; ++q) idx[a][q] = min(max(c[a] + OFF + q, 0), v.n[a] - 1);
      contract([&](int i, int j, float (&sv)[K]) {
        const float* row = v.v + ((int64_t)idx[0][i] * v.n[1] + idx[1][j]) * (int64_t)v.n[2];
#pragma unroll
        for (int k = 0; k < K; ++k) sv[k] = row[idx[2][k]];
      });
    }
    return make_float4(f, fx * v.inv_h[0], fy * v.inv_h[1], fz * v.inv_h[2]);
  }
}

// Four lanes per ray, as in the model renderer: a wave holds a 4x4 pixel
// tile, lane s of a ray's group evaluates samples s, s + 4, ..., and the
// group composites its four shaded samples in ray order with the
// operations of one lane stepping through them (a sample past the end of
// the ray enters with opacity 0, which leaves the pixel exactly unchanged),
// stopping at the same sample.
template <int KIND>
__global__ __launch_bounds__(kBlock) void volume_k(VolArgs v, RenderArgs r) {
  __shared__ float4 tf[256];
  __shared__ int zpre[257];
  __shared__ int wtot[kBlock / kWave];
  stage_tf(r.tf, tf, zpre, wtot);
  const int tx = (r.w + 7) / 8, ty = (r.h + 7) / 8;
  const int tile = frame_tile(blockIdx.x, tx, ty);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, s = lane & 3;
  const int i = (tile % tx) * 8 + (wave & 1) * 4 + ((lane >> 2) & 3);
  const int j = (tile / tx) * 8 + (wave >> 1) * 4 + (lane >> 4);
  const bool pix = i < r.w && j < r.h;
  Ray ray;
  ray.K = 0;
  if (pix) ray = make_ray_box(v.lo, v.hi, r, i, j);
  float L[3] = {0.f, 0.f, 0.f};
  if (pix) {
    const double dn = sqrt(ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) L[a] = (float)(-ray.d[a] / dn);
  }
  const int64_t pid = (int64_t)j * r.w + i;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
  int used = 0;
  bool done = false;
  for (int kb = 0;; kb += 4) {
    const bool act = pix && !done && kb < ray.K;     // the same in the four lanes of a ray
    if (__ballot(act) == 0) break;                 // whole wave finished
    if (!act) continue;
    const int k = kb + s;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < ray.K) {
      double x[3];
      sample_point(ray, r.step, k, x);
      q = shade_sample(volume_field<KIND>(v, x), L, tf, r);
    }
    const float4 q0 = quad_bcast4<0>(q), q1 = quad_bcast4<1>(q), q2 = quad_bcast4<2>(q),
                 q3 = quad_bcast4<3>(q);
    int stop = 0;                  // 1 + index of the terminating sample, 0: none
    auto step = [&](float4 qt, int t) {
      const bool live = stop == 0;
      qt.w = live ? qt.w : 0.f;
      over(qt, C0, C1, C2, A);
      if (live && A >= r.ert_alpha) stop = t + 1;
    };
    step(q0, 0);
    step(q1, 1);
    step(q2, 2);
    step(q3, 3);
    done = stop != 0;
    used = done ? kb + stop : min(kb + 4, ray.K);
    if (r.alpha && k < used) r.alpha[pid * r.alpha_stride + k] = q.w;
  }
  if (pix && s == 0) {
    reinterpret_cast<float4*>(r.rgba)[pid] = make_float4(C0, C1, C2, A);
    if (r.nsamp) reinterpret_cast<int2*>(r.nsamp)[pid] = make_int2(ray.K, used);
    if (r.neval) r.neval[pid] = used;
  }
}

// ------------------------------------------------------------------ K6: persistent serving
// Each workgroup takes work items from an atomic cursor until the batch is
// exhausted (every wave reaches the exit once the cursor passes n_items).
// The kernel instance fixes (degree, storage, multi-block); requests of one
// batch may use any model of that kind and any mix of frames and query sets.
template <int P, Storage S, bool MULTI>
__global__ __launch_bounds__(kBlock) void serve_k(const DevModel* __restrict__ models,
                                                  const ServeReq* __restrict__ reqs,
                                                  const ServeItem* __restrict__ items, int n_items,
                                                  int* __restrict__ cursor) {
  __shared__ float4 tf[256];
  __shared__ int zpre[257];
  __shared__ int wtot[kBlock / kWave];
  __shared__ int s_item;
  int staged = -1;                                 // request whose TF is in LDS
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(cursor, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) return;
    const ServeItem I = items[it];
    const ServeReq* Q = reqs + I.req;
    const DevModel& m = models[Q->model];
    if (Q->kind == kServeRender) {
      if (staged != I.req) {
        stage_tf(Q->ra.tf, tf, zpre, wtot);
        staged = I.req;
      }
      render_tile<P, S, MULTI>(m, Q->ra, I.index, m.rec, m.mats, tf, zpre, m.edges);
      __syncthreads();                             // tf may be restaged by the next item
    } else {
      const int64_t i = (int64_t)I.index * kBlock + threadIdx.x;
      if (i < Q->n) {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(m.ctrl, m.ctrl_bytes);
        const double x[3] = {(double)Q->xyz[i], (double)Q->xyz[Q->n + i], (double)Q->xyz[2 * Q->n + i]};
        const Loc L = locate<P, MULTI>(m, m.rec, x);
        reinterpret_cast<float4*>(Q->out)[i] = evaluate<P, S, !MULTI>(L, rs, m.mats, m.mat_stride, m.imat);
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
// Span records and tables go to LDS when they fit this budget (non-uniform
// knots give every span its own basis table: 128 spans per axis take about
// 54 KB); with the decode window (at most 32 KB) a workgroup stays within
// the 160 KB of LDS of a CU.
constexpr int kLdsRecBytes = 64 * 1024;
constexpr size_t kStaticLdsBytes = 8 * 1024;   // a kernel's own LDS arrays, at most

// Whether dyn bytes of dynamic LDS (plus the kernel's own arrays) fit a
// workgroup on the current device (its limit read once per device).
static bool lds_fits(size_t dyn) {
  static std::atomic<int> limit[64];     // zero-initialised: not read yet
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return dyn + kStaticLdsBytes <= 65536;
  int v = limit[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 65536;
    limit[dev].store(v, std::memory_order_relaxed);
  }
  return dyn + kStaticLdsBytes <= (size_t)v;
}

template <int P, Storage S, bool G>
static void points_g(const DevModel& m, int kind, const float* xyz, int64_t n, float* out,
                     int32_t* dbg, hipStream_t st) {
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  if (kind == kKindMulti)
    hipLaunchKernelGGL((decode_points_k<P, S, true, false, G>), dim3(grid), dim3(kBlock), 0, st, m,
                       xyz, n, out, dbg);
  else if (kind == kKindGraded)
    hipLaunchKernelGGL((decode_points_k<P, S, false, true, G>), dim3(grid), dim3(kBlock), 0, st, m,
                       xyz, n, out, dbg);
  else
    hipLaunchKernelGGL((decode_points_k<P, S, false, false, G>), dim3(grid), dim3(kBlock), 0, st, m,
                       xyz, n, out, dbg);
}

template <int P, Storage S>
static hipError_t points_p(const DevModel& m, int kind, bool grad, const float* xyz, int64_t n,
                           float* out, int32_t* dbg, hipStream_t st) {
  if (grad)
    points_g<P, S, true>(m, kind, xyz, n, out, dbg, st);
  else
    points_g<P, S, false>(m, kind, xyz, n, out, dbg, st);
  return hipGetLastError();
}

// Histogram, scan and scatter of the (block, tile) sort.
template <bool MULTI, bool GT, bool TL>
static void sort_launch_tl(const DevModel& m, const SortArgs& sa, size_t tabs, hipStream_t st) {
  // a chunk per workgroup, at most kHistGrid workgroups (each then takes
  // several chunks: fewer final additions to the global counts)
  const unsigned gh =
      (unsigned)std::min<int64_t>((sa.n + hist_chunk<MULTI>() - 1) / hist_chunk<MULTI>(), kHistGrid);
  const size_t hist_lds = tabs + (size_t)((sa.nb + 1) / 2) * 4;
  hipLaunchKernelGGL((sort_hist_k<MULTI, GT, TL>), dim3(gh), dim3(kHistThreads), hist_lds, st, m, sa);
  hipLaunchKernelGGL(sort_scan_k, dim3(1), dim3(kScanThreads), 0, st, sa);
  // at most 8 workgroups per CU, each looping over chunks; a multiple of 8
  // (the chunk bands of sort_scatter_k)
  const unsigned gc = ((unsigned)std::min<int64_t>((sa.n + kScatterChunk - 1) / kScatterChunk, 8 * 256) +
                       7u) & ~7u;
  if (sa.bkt) {                        // two levels, buckets from the histogram pass
    hipLaunchKernelGGL((sort_scatter_k<false, kCoarse, false, false, true>), dim3(gc), dim3(kBlock), 0, st,
                       m, sa);
    hipLaunchKernelGGL((sort_scatter_k<false, kFine, false, false, true>), dim3(gc), dim3(kBlock), 0, st,
                       m, sa);
  } else if (sa.tmp) {                 // two levels: coarse runs, then buckets
    hipLaunchKernelGGL((sort_scatter_k<MULTI, kCoarse, GT, TL>), dim3(gc), dim3(kBlock), tabs, st, m, sa);
    hipLaunchKernelGGL((sort_scatter_k<MULTI, kFine, GT, TL>), dim3(gc), dim3(kBlock), tabs, st, m, sa);
  } else {
    hipLaunchKernelGGL((sort_scatter_k<MULTI, kOne, GT, TL>), dim3(gc), dim3(kBlock), tabs, st, m, sa);
  }
}

template <bool MULTI, bool GT>
static void sort_launch(const DevModel& m, const SortArgs& sa, hipStream_t st) {
  if constexpr (MULTI) {
    const size_t tabs = sort_tabs_bytes<MULTI>(m);
    if (tabs != 0)
      sort_launch_tl<MULTI, GT, true>(m, sa, tabs, st);
    else
      sort_launch_tl<MULTI, GT, false>(m, sa, 0, st);
  } else {
    sort_launch_tl<MULTI, GT, false>(m, sa, 0, st);
  }
}

template <int P, Storage S, bool G>
static void decode_sorted_g(const DevModel& m, int kind, const SortArgs& sa, float* out,
                            int32_t* dbg, hipStream_t st) {
  const size_t tabs = (size_t)m.n_rec * sizeof(SpanRec) + (size_t)m.n_mats * m.mat_stride * 4;
  const size_t wb = (size_t)m.win_max * 4;
  const bool lds_tabs = tabs <= (size_t)kLdsRecBytes && lds_fits(tabs + wb);
  const bool ldsrec = kind != kKindMulti && lds_tabs;     // span records and tables staged together
  // windows too large for LDS, or basis tables too large for the LDS copy
  // of the kernels that stage the windows alone: one point per thread
  if (m.win_max > kWinMax || (!ldsrec && m.n_mats * m.mat_stride > kMatsLds)) {
    const unsigned g = (unsigned)((sa.n + kBlock - 1) / kBlock);
    if (kind != kKindPlain)
      hipLaunchKernelGGL((decode_sorted_k<P, S, true, false, G>), dim3(g), dim3(kBlock), 0, st, m, sa,
                         out, dbg);
    else
      hipLaunchKernelGGL((decode_sorted_k<P, S, false, false, G>), dim3(g), dim3(kBlock), 0, st, m, sa,
                         out, dbg);
    return;
  }
  // items: at most ceil(n / kTilePoints) + nb; the surplus workgroups exit
  const unsigned gi = (unsigned)((sa.n + kTilePoints - 1) / kTilePoints + sa.nb);
  const int cap = m.win_max;
  if (kind == kKindMulti || (kind == kKindGraded && !lds_tabs))
    hipLaunchKernelGGL((decode_tiles_k<P, S, true, false, false, G>), dim3(gi), dim3(kBlock), wb, st, m,
                       sa, cap, out, dbg);
  else if (kind == kKindGraded)
    hipLaunchKernelGGL((decode_tiles_k<P, S, false, true, true, G>), dim3(gi), dim3(kBlock), tabs + wb,
                       st, m, sa, cap, out, dbg);
  else if (lds_tabs)
    hipLaunchKernelGGL((decode_tiles_k<P, S, false, true, false, G>), dim3(gi), dim3(kBlock), tabs + wb,
                       st, m, sa, cap, out, dbg);
  else
    hipLaunchKernelGGL((decode_tiles_k<P, S, false, false, false, G>), dim3(gi), dim3(kBlock), wb, st, m,
                       sa, cap, out, dbg);
}

// Results of the decode in coarse order (sa.tpos) gathered back into input
// order: out[i] = src[tpos[i]].  The positions of consecutive points fall
// into one short run per coarse key of their scatter chunk, so the gathers
// read whole lines.  tpos is read once and out written once in whole
// lines: streaming loads and stores.
constexpr int kUnsortPer = 4;

template <bool G>
__global__ __launch_bounds__(kBlock) void unsort_k(const uint32_t* __restrict__ tpos,
                                                   const float* __restrict__ src, int64_t n,
                                                   float* __restrict__ out) {
  // every load is unconditional (indices clamped into range) so that all
  // of a thread's loads are in flight together; only the stores are masked
  const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kUnsortPer) + threadIdx.x;
  uint32_t k[kUnsortPer];
#pragma unroll
  for (int u = 0; u < kUnsortPer; ++u)
    k[u] = min(__builtin_nontemporal_load(tpos + min(i0 + u * kBlock, n - 1)), (uint32_t)(n - 1));
  // A slot past n repeats element n - 1 (its tpos entry, its value and its
  // destination), a duplicate write of an equal value.  The empty asm takes
  // all gathered values before the first store, so no store is in flight
  // while the loads are waited for.
  if constexpr (G) {
    f32x4 v[kUnsortPer];
#pragma unroll
    for (int u = 0; u < kUnsortPer; ++u) v[u] = reinterpret_cast<const f32x4*>(src)[k[u]];
    static_assert(kUnsortPer == 4, "one asm operand per value");
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]) : : "memory");
#pragma unroll
    for (int u = 0; u < kUnsortPer; ++u)
      __builtin_nontemporal_store(v[u], reinterpret_cast<f32x4*>(out) + min(i0 + u * kBlock, n - 1));
  } else {
    float v[kUnsortPer];
#pragma unroll
    for (int u = 0; u < kUnsortPer; ++u) v[u] = src[k[u]];
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]) : : "memory");
#pragma unroll
    for (int u = 0; u < kUnsortPer; ++u) __builtin_nontemporal_store(v[u], out + min(i0 + u * kBlock, n - 1));
  }
}

template <int P, Storage S>
static hipError_t sorted_p(const DevModel& m, int kind, bool grad, const SortArgs& sa, float* out,
                           int32_t* dbg, hipStream_t st) {
  const bool multi = kind == kKindMulti;
  const unsigned gb = (unsigned)((sa.nb + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(fill_u32_k, dim3(gb), dim3(kBlock), 0, st, sa.hist, (int64_t)sa.nb);
  if (multi)
    sort_launch<true, false>(m, sa, st);
  else if (kind == kKindGraded)
    sort_launch<false, true>(m, sa, st);
  else
    sort_launch<false, false>(m, sa, st);
  float* dout = sa.tpos ? reinterpret_cast<float*>(sa.tmp) : out;
  if (grad)
    decode_sorted_g<P, S, true>(m, kind, sa, dout, dbg, st);
  else
    decode_sorted_g<P, S, false>(m, kind, sa, dout, dbg, st);
  if (sa.tpos) {
    const unsigned g = (unsigned)((sa.n + kBlock * kUnsortPer - 1) / (kBlock * kUnsortPer));
    if (grad)
      hipLaunchKernelGGL(unsort_k<true>, dim3(g), dim3(kBlock), 0, st, sa.tpos, dout, sa.n, out);
    else
      hipLaunchKernelGGL(unsort_k<false>, dim3(g), dim3(kBlock), 0, st, sa.tpos, dout, sa.n, out);
  }
  return hipGetLastError();
}

template <int P, Storage S>
static hipError_t serve_p(bool multi, const DevModel* models, const ServeReq* reqs,
                          const ServeItem* items, int n_items, int* cursor, int grid, hipStream_t st) {
  if (multi)
    hipLaunchKernelGGL((serve_k<P, S, true>), dim3(grid), dim3(kBlock), 0, st, models, reqs, items,
                       n_items, cursor);
  else
    hipLaunchKernelGGL((serve_k<P, S, false>), dim3(grid), dim3(kBlock), 0, st, models, reqs, items,
                       n_items, cursor);
  return hipGetLastError();
}

template <int P, Storage S>
static hipError_t grid_p(const DevModel& m, bool grad, GridArgs ga, hipStream_t st) {
  ga.ta = kGridTA;
  dim3 grid((ga.res[2] + kWave - 1) / kWave, (ga.res[1] + 3) / 4, (ga.res[0] + kGridTA - 1) / kGridTA);
  if (grad)
    hipLaunchKernelGGL((decode_grid_k<P, S, true>), grid, dim3(kBlock), 0, st, m, ga);
  else
    hipLaunchKernelGGL((decode_grid_k<P, S, false>), grid, dim3(kBlock), 0, st, m, ga);
  return hipGetLastError();
}

template <int P, Storage S>
static hipError_t render_p(const DevModel& m, int kind, const RenderArgs& r, hipStream_t st) {
  const int tiles = ((r.w + kTile - 1) / kTile) * ((r.h + kTile - 1) / kTile);
  const int tiles8 = ((r.w + 7) / 8) * ((r.h + 7) / 8);     // four lanes per ray
  const size_t lds = (size_t)m.n_rec * sizeof(SpanRec) + (size_t)m.n_mats * m.mat_stride * 4;
  // a single block with a non-uniform axis: its own kernel when the tables
  // fit in LDS, else the multi-block kernels
  const bool lds_tabs = lds <= (size_t)kLdsRecBytes && lds_fits(lds);
  const bool multi = kind == kKindMulti || (kind == kKindGraded && !lds_tabs);
  const bool gm = m.n_mats * m.mat_stride > kMatsLds;    // basis tables beyond the LDS copy
  // a partial render of a single-block model holds every sample (its
  // region is the model box): it is the full render, whose key is the
  // entry parameter of the model box
  if ((multi || !lds_tabs) && gm && r.partial)
    hipLaunchKernelGGL((render_k<P, S, true, false, true, false, false, true>), dim3(tiles), dim3(kBlock),
                       0, st, m, r);
  else if ((multi || !lds_tabs) && gm)
    hipLaunchKernelGGL((render_k<P, S, true, false, false, false, false, true>), dim3(tiles), dim3(kBlock),
                       0, st, m, r);
  else if (multi && r.partial)
    hipLaunchKernelGGL((render_k<P, S, true, false, true>), dim3(tiles), dim3(kBlock), 0, st, m, r);
  else if (multi && m.n_edges <= kEdgesLds)   // one lane per ray (four per ray measured slower here)
    hipLaunchKernelGGL((render_k<P, S, true, false, false, false, false, false, true>), dim3(tiles),
                       dim3(kBlock), 0, st, m, r);
  else if (multi)
    hipLaunchKernelGGL((render_k<P, S, true, false>), dim3(tiles), dim3(kBlock), 0, st, m, r);
  else if (kind == kKindGraded && r.partial)
    hipLaunchKernelGGL((render_k<P, S, false, true, false, true>), dim3(tiles), dim3(kBlock), lds, st,
                       m, r);
  else if (kind == kKindGraded)
    hipLaunchKernelGGL((render_k<P, S, false, true, false, true, true>), dim3(tiles8), dim3(kBlock), lds,
                       st, m, r);
  else if (lds_tabs && r.partial)
    hipLaunchKernelGGL((render_k<P, S, false, true>), dim3(tiles), dim3(kBlock), lds, st, m, r);
  else if (lds_tabs)
    hipLaunchKernelGGL((render_k<P, S, false, true, false, false, true>), dim3(tiles8), dim3(kBlock), lds,
                       st, m, r);
  else if (r.partial)
    hipLaunchKernelGGL((render_k<P, S, false, false>), dim3(tiles), dim3(kBlock), 0, st, m, r);
  else
    hipLaunchKernelGGL((render_k<P, S, false, false, false, false, true>), dim3(tiles8), dim3(kBlock), 0,
                       st, m, r);
  return hipGetLastError();
}

template <int P, Storage S>
static hipError_t iso_p(const DevModel& m, int kind, const RenderArgs& r, hipStream_t st) {
  const int tiles = ((r.w + kTile - 1) / kTile) * ((r.h + kTile - 1) / kTile);
  const int tiles8 = ((r.w + 7) / 8) * ((r.h + 7) / 8);
  const size_t lds = (size_t)m.n_rec * sizeof(SpanRec) + (size_t)m.n_mats * m.mat_stride * 4;
  const bool lds_tabs = lds <= (size_t)kLdsRecBytes && lds_fits(lds);
  if (kind == kKindMulti || (kind == kKindGraded && !lds_tabs))
    hipLaunchKernelGGL((iso_k<P, S, true, false>), dim3(tiles), dim3(kBlock), 0, st, m, r);
  else if (kind == kKindGraded)        // four lanes per ray
    hipLaunchKernelGGL((iso_k<P, S, false, true, true, true>), dim3(tiles8), dim3(kBlock), lds, st, m, r);
  else if (lds_tabs)
    hipLaunchKernelGGL((iso_k<P, S, false, true, false, true>), dim3(tiles8), dim3(kBlock), lds, st, m, r);
  else
    hipLaunchKernelGGL((iso_k<P, S, false, false>), dim3(tiles), dim3(kBlock), 0, st, m, r);
  return hipGetLastError();
}

#define MFA_DISPATCH(FN, ...)                                                        \
  switch (p) {                                                                       \
    case 1: return s == Storage::F32 ? FN<1, Storage::F32>(__VA_ARGS__)              \
                 : s == Storage::BF16 ? FN<1, Storage::BF16>(__VA_ARGS__)            \
                                      : FN<1, Storage::F16>(__VA_ARGS__);            \
    case 2: return s == Storage::F32 ? FN<2, Storage::F32>(__VA_ARGS__)              \
                 : s == Storage::BF16 ? FN<2, Storage::BF16>(__VA_ARGS__)            \
                                      : FN<2, Storage::F16>(__VA_ARGS__);            \
    case 3: return s == Storage::F32 ? FN<3, Storage::F32>(__VA_ARGS__)              \
                 : s == Storage::BF16 ? FN<3, Storage::BF16>(__VA_ARGS__)            \
                                      : FN<3, Storage::F16>(__VA_ARGS__);            \
    case 4: return s == Storage::F32 ? FN<4, Storage::F32>(__VA_ARGS__)              \
                 : s == Storage::BF16 ? FN<4, Storage::BF16>(__VA_ARGS__)            \
                                      : FN<4, Storage::F16>(__VA_ARGS__);            \
    case 5: return s == Storage::F32 ? FN<5, Storage::F32>(__VA_ARGS__)              \
                 : s == Storage::BF16 ? FN<5, Storage::BF16>(__VA_ARGS__)            \
                                      : FN<5, Storage::F16>(__VA_ARGS__);            \
    default: return hipErrorInvalidValue;                                            \
  }

hipError_t launch_decode_points(const DevModel& m, int p, Storage s, int kind, bool grad,
                                const float* xyz, int64_t n, float* out, int32_t* dbg,
                                hipStream_t st) {
  MFA_DISPATCH(points_p, m, kind, grad, xyz, n, out, dbg, st)
}

hipError_t launch_decode_sorted(const DevModel& m, int p, Storage s, int kind, bool grad,
                                const SortArgs& sa, float* out, int32_t* dbg, hipStream_t st) {
  MFA_DISPATCH(sorted_p, m, kind, grad, sa, out, dbg, st)
}

hipError_t launch_serve(int p, Storage s, bool multi, const DevModel* models, const ServeReq* reqs,
                        const ServeItem* items, int n_items, int* cursor, int grid, hipStream_t st) {
  MFA_DISPATCH(serve_p, multi, models, reqs, items, n_items, cursor, grid, st)
}

// Scratch of the allocation-free sorted decode: a file-scope device array
// (each device holding its own copy until the process ends).  Host code
// never passes the array's name to a kernel: on the host it is a stand-in,
// not a device address.  The device address is read once per device, with
// that device current, by hipGetSymbolAddress and kept here.
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::atomic<void*> addr[kMaxDevices];
  static std::mutex mu;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* a = addr[dev].load(std::memory_order_acquire);
  if (a == nullptr) {
    std::lock_guard<std::mutex> g(mu);
    a = addr[dev].load(std::memory_order_relaxed);
    if (a == nullptr) {
      e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      if (a == nullptr) return hipErrorInvalidSymbol;
      addr[dev].store(a, std::memory_order_release);
    }
  }
  *ptr = a;
  return hipSuccess;
}

hipError_t launch_decode_grid(const DevModel& m, int p, Storage s, bool grad, const GridArgs& ga,
                              hipStream_t st) {
  MFA_DISPATCH(grid_p, m, grad, ga, st)
}

hipError_t launch_render(const DevModel& m, int p, Storage s, int kind, const RenderArgs& r,
                         hipStream_t st) {
  MFA_DISPATCH(render_p, m, kind, r, st)
}

hipError_t launch_iso(const DevModel& m, int p, Storage s, int kind, const RenderArgs& r,
                      hipStream_t st) {
  MFA_DISPATCH(iso_p, m, kind, r, st)
}

hipError_t launch_volume(const VolArgs& v, int kind, const RenderArgs& r, hipStream_t st) {
  const int tiles = ((r.w + 7) / 8) * ((r.h + 7) / 8);     // 8x8 pixels, four lanes per ray
  switch (kind) {
    case MFA_FILTER_TRILINEAR:
      hipLaunchKernelGGL(volume_k<MFA_FILTER_TRILINEAR>, dim3(tiles), dim3(kBlock), 0, st, v, r);
      break;
    case MFA_FILTER_CATMULL_ROM:
      hipLaunchKernelGGL(volume_k<MFA_FILTER_CATMULL_ROM>, dim3(tiles), dim3(kBlock), 0, st, v, r);
      break;
    case MFA_FILTER_CUBIC_BSPLINE:
      hipLaunchKernelGGL(volume_k<MFA_FILTER_CUBIC_BSPLINE>, dim3(tiles), dim3(kBlock), 0, st, v, r);
      break;
    case MFA_FIELD_MARSCHNER_LOBB:
      hipLaunchKernelGGL(volume_k<MFA_FIELD_MARSCHNER_LOBB>, dim3(tiles), dim3(kBlock), 0, st, v, r);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ K7: compositing
// Depth-ordered "over" of partial images (Sec. IV-A5: compositing relies on
// the associativity of the operator, in depth order).  One thread per pixel:
// the pixel of every partial is loaded first (coalesced 16-byte reads, in
// list order), the (key, colour) tuples are sorted in registers by an
// odd-even transposition network over GMAX slots (GMAX the smallest of 2, 4,
// 8, 16 holding the G partials; unused slots hold +inf and sort last; a
// swap needs a strictly smaller key, so equal keys keep list order), then
// folded front to back: C += (1 - A) c, A += (1 - A) a.  Reads 24 bytes per
// partial and writes 16 per pixel: HBM-bound.
template <int GMAX>
__global__ __launch_bounds__(kBlock) void composite_k(CompositeArgs c) {
  const int64_t px = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (px >= c.npix) return;
  double kv[GMAX];
  float4 v[GMAX];
#pragma unroll
  for (int g = 0; g < GMAX; ++g) {
    if (g < c.g) {
      kv[g] = c.keys[g][px];
      v[g] = c.images[g][px];
    } else {
      kv[g] = __builtin_inf();
      v[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int round = 0; round < GMAX; ++round) {
#pragma unroll
    for (int g = round & 1; g + 1 < GMAX; g += 2) {
      if (kv[g + 1] < kv[g]) {                 // adjacent transposition keeps ties stable
        const double tk = kv[g];
        kv[g] = kv[g + 1];
        kv[g + 1] = tk;
        const float4 tv = v[g];
        v[g] = v[g + 1];
        v[g + 1] = tv;
      }
    }
  }
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
#pragma unroll
  for (int g = 0; g < GMAX; ++g) {
    const float om = 1.f - A;
    C0 = fmaf(om, v[g].x, C0);
    C1 = fmaf(om, v[g].y, C1);
    C2 = fmaf(om, v[g].z, C2);
    A = fmaf(om, v[g].w, A);
  }
  store_stream(&c.out[px], make_float4(C0, C1, C2, A));
}

hipError_t launch_composite(const CompositeArgs& c, hipStream_t st) {
  const int64_t blocks = (c.npix + kBlock - 1) / kBlock;
  if (blocks == 0) return hipSuccess;
  if (c.g <= 2)
    hipLaunchKernelGGL(composite_k<2>, dim3((unsigned)blocks), dim3(kBlock), 0, st, c);
  else if (c.g <= 4)
    hipLaunchKernelGGL(composite_k<4>, dim3((unsigned)blocks), dim3(kBlock), 0, st, c);
  else if (c.g <= 8)
    hipLaunchKernelGGL(composite_k<8>, dim3((unsigned)blocks), dim3(kBlock), 0, st, c);
  else
    hipLaunchKernelGGL(composite_k<16>, dim3((unsigned)blocks), dim3(kBlock), 0, st, c);
  return hipGetLastError();
}

}  // namespace mfa
