// Host side of the MFA library: argument validation, the model store
// (storage rounding, knot-span records, per-span basis polynomials, block
// table, upload) and the C entry points that enqueue the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "mfa.h"
#include "mfa_internal.h"
#include "mfa_model.h"

namespace mfa {
hipError_t launch_decode_points(const DevModel& m, int p, Storage s, int kind, bool grad,
                                const float* xyz, int64_t n, float* out, int32_t* dbg,
                                hipStream_t st);
hipError_t launch_decode_grid(const DevModel& m, int p, Storage s, bool grad, const GridArgs& ga,
                              hipStream_t st);
hipError_t launch_decode_sorted(const DevModel& m, int p, Storage s, int kind, bool grad,
                                const SortArgs& sa, float* out, int32_t* dbg, hipStream_t st);
hipError_t static_scratch(void** ptr);
hipError_t launch_render(const DevModel& m, int p, Storage s, int kind, const RenderArgs& r,
                         hipStream_t st);
hipError_t launch_composite(const CompositeArgs& c, hipStream_t st);
hipError_t launch_iso(const DevModel& m, int p, Storage s, int kind, const RenderArgs& r,
                      hipStream_t st);
hipError_t launch_volume(const VolArgs& v, int kind, const RenderArgs& r, hipStream_t st);
}  // namespace mfa

using namespace mfa;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

mfa_status fail(mfa_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

mfa_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? MFA_E_NOMEM : MFA_E_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

// ------------------------------------------------------------------ storage rounding
// FP64 -> FP32 is the C++ conversion (round to nearest even).  FP32 ->
// BF16 keeps the top half after adding 0x7FFF plus the lowest kept bit;
// FP32 -> FP16 rounds the significand to 11 bits with gradual underflow.
static uint32_t f32_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

static uint16_t to_bf16(float f) {
  const uint32_t u = f32_bits(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
    return (uint16_t)((u >> 16) | 0x0040u);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

static uint16_t to_f16(float f) {
  const uint32_t u = f32_bits(f);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const int32_t exp = (int32_t)((u >> 23) & 0xFF);
  const uint32_t man = u & 0x7FFFFFu;
  if (exp == 0xFF) return (uint16_t)(sign | 0x7C00u | (man ? 0x200u | (man >> 13) : 0u));
  const int32_t e16 = exp - 127 + 15;
  if (e16 >= 31) return (uint16_t)(sign | 0x7C00u);
  uint32_t sig = exp ? (man | 0x800000u) : man;
  int shift = e16 >= 1 ? 13 : 14 - e16;
  if (exp == 0 || shift > 25) return (uint16_t)sign;      // below half the smallest subnormal
  uint32_t kept = sig >> shift;
  const uint32_t rem = sig & ((1u << shift) - 1u);
  const uint32_t half = 1u << (shift - 1);
  if (rem > half || (rem == half && (kept & 1u))) ++kept;
  uint32_t mag = e16 >= 1 ? ((uint32_t)e16 << 10) + (kept - 0x400u) : kept;
  if (mag >= 0x7C00u) mag = 0x7C00u;
  return (uint16_t)(sign | mag);
}

static float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static float f16_value(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const uint32_t exp = (h >> 10) & 0x1F, man = h & 0x3FFu;
  float v;
  if (exp == 0) v = std::ldexp((float)man, -24);
  else if (exp == 31) v = man ? NAN : INFINITY;
  else v = std::ldexp((float)(man | 0x400u), (int)exp - 25);
  uint32_t u = f32_bits(v) | sign;
  std::memcpy(&v, &u, 4);
  return v;
}

static int elem_size(mfa_dtype d) { return d == MFA_F32 ? 4 : 2; }

// FP16 pattern of the largest half <= v (down) or smallest half >= v (up);
// beyond the half range the result is the corresponding infinity.
static uint16_t f16_directed(float v, bool up) {
  uint16_t h = to_f16(v);
  const float hv = f16_value(h);
  if (up ? hv >= v : hv <= v) return h;
  // step one ulp in the needed direction (sign-magnitude encoding)
  const bool neg = (h & 0x8000u) != 0;
  if ((h & 0x7FFFu) == 0) return up ? 0x0001u : 0x8001u;     // +-0 -> +-smallest subnormal
  const bool away = up != neg;            // moving away from zero?
  return (uint16_t)(away ? h + 1 : h - 1);
}

// ------------------------------------------------------------------ basis polynomials
// Pieces of the degree-p basis functions active on span s as polynomials in
// tau = (u - T[s]) / h: the Cox-de Boor recursion applied to polynomials,
// with u = T[s] + h tau substituted into each linear weight (FP64), then
// rounded to FP32.  Layout: see mat_stride().
static std::vector<float> span_table(const double* T, int p, int s) {
  const double ts = T[s], h = T[s + 1] - T[s];
  std::vector<std::vector<double>> N(1, std::vector<double>(p + 1, 0.0));
  N[0][0] = 1.0;
  for (int q = 1; q <= p; ++q) {
    std::vector<std::vector<double>> M(q + 1, std::vector<double>(p + 1, 0.0));
    for (int r = 0; r <= q; ++r) {
      const int i = s - q + r;
      if (r >= 1) {
        const double den = T[i + q] - T[i];
        if (den != 0.0) {
          const double a0 = (ts - T[i]) / den, a1 = h / den;   // (u - T_i)/den
          for (int m = 0; m <= p; ++m) {
            M[r][m] += a0 * N[r - 1][m];
            if (m + 1 <= p) M[r][m + 1] += a1 * N[r - 1][m];
          }
        }
      }
      if (r <= q - 1) {
        const double den = T[i + q + 1] - T[i + 1];
        if (den != 0.0) {
          const double b0 = (T[i + q + 1] - ts) / den, b1 = -h / den;  // (T_{i+q+1} - u)/den
          for (int m = 0; m <= p; ++m) {
            M[r][m] += b0 * N[r][m];
            if (m + 1 <= p) M[r][m + 1] += b1 * N[r][m];
          }
        }
      }
    }
    N.swap(M);
  }
  std::vector<float> out(mat_stride(p), 0.f);
  for (int r = 0; r <= p; ++r)
    for (int m = 0; m <= p; ++m) out[r * (p + 1) + m] = (float)N[r][m];
  for (int r = 0; r <= p; ++r)
    for (int m = 0; m < p; ++m) out[(p + 1) * (p + 1) + r * p + m] = (float)((m + 1) * N[r][m + 1]);
  return out;
}

// The uniform interior table of degree p as a vector (see UniformTable).
template <int P>
static std::vector<float> uniform_table_p() {
  constexpr UniformTable<P> U{};
  return std::vector<float>(U.c, U.c + mat_stride(P));
}

static std::vector<float> uniform_table(int p) {
  switch (p) {
    case 1: return uniform_table_p<1>();
    case 2: return uniform_table_p<2>();
    case 3: return uniform_table_p<3>();
    case 4: return uniform_table_p<4>();
    case 5: return uniform_table_p<5>();
    default: return {};
  }
}

// Equal to the canonical table up to FP64 rounding of the knots: within
// 1e-6 of its largest coefficient, entry by entry (tables of other span
// shapes differ by O(0.1)).
static bool near_table(const std::vector<float>& a, const std::vector<float>& b) {
  if (a.size() != b.size()) return false;
  float scale = 0.f;
  for (float v : b) scale = std::max(scale, std::fabs(v));
  for (size_t q = 0; q < a.size(); ++q)
    if (!(std::fabs(a[q] - b[q]) <= 1e-6f * scale)) return false;
  return true;
}

// ------------------------------------------------------------------ model

static void free_model(mfa_model m) {
  if (!m) return;
  if (m->ws_done) (void)hipEventDestroy(m->ws_done);
  void* bufs[] = {m->d_ctrl, m->d_rec, m->d_mats, m->d_blocks, m->d_edges, m->d_mcb, m->d_scb[0], m->d_scb[1], m->d_bwin, m->d_gtab, m->d_gmeta, m->d_ws, m->d_sblk, m->d_sedges};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete m;
}

static bool is_fin(double v) { return std::isfinite(v); }

mfa_status check_knots(const double* T, int n, int p, int blk, int axis) {
  for (int i = 0; i < n + p + 1; ++i)
    if (!is_fin(T[i])) return fail(MFA_E_ARG, "block %d axis %d: knot %d not finite", blk, axis, i);
  for (int i = 0; i + 1 < n + p + 1; ++i)
    if (T[i + 1] < T[i]) return fail(MFA_E_ARG, "block %d axis %d: knots decrease at %d", blk, axis, i);
  for (int i = 0; i <= p; ++i)
    if (T[i] != 0.0 || T[n + i] != 1.0)
      return fail(MFA_E_ARG, "block %d axis %d: knots must be clamped to [0,1] (p+1 end knots)", blk,
                  axis);
  if (!(T[n - 1] < 1.0))
    return fail(MFA_E_ARG, "block %d axis %d: last span [T[n-1], T[n]] is empty", blk, axis);
  return MFA_OK;
}

void default_knots(int n, int p, double* T) {
  for (int i = 0; i <= p; ++i) {
    T[i] = 0.0;
    T[n + i] = 1.0;
  }
  const double nsp = (double)(n - p);
  for (int j = 1; j < n - p; ++j) T[p + j] = (double)j / nsp;
}

// Value bounds per macro cell (2^shift spans per axis) of one block: min and max of
// the stored control points that act on any span of the cell (the spline is
// a convex combination of them), by windowed min/max one axis at a time.
static void macro_bounds(const std::vector<float>& V, const int n[3], int p, int shift,
                         const int mc[3], std::vector<float2>& out) {
  const int mk = 1 << shift;
  auto win = [&](int a, int c, int& lo, int& hi) {
    lo = c * mk;
    hi = std::min(c * mk + mk - 1, n[a] - p - 1) + p;
  };
  const int n0 = n[0], n1 = n[1], n2 = n[2];
  std::vector<float> lo2((size_t)n0 * n1 * mc[2]), hi2(lo2.size());
  for (int64_t r = 0; r < (int64_t)n0 * n1; ++r)
    for (int c = 0; c < mc[2]; ++c) {
      int a0, a1;
      win(2, c, a0, a1);
      float mn = INFINITY, mx = -INFINITY;
      for (int k = a0; k <= a1; ++k) {
        mn = std::fmin(mn, V[r * n2 + k]);
        mx = std::fmax(mx, V[r * n2 + k]);
      }
      lo2[r * mc[2] + c] = mn;
      hi2[r * mc[2] + c] = mx;
    }
  std::vector<float> lo1((size_t)n0 * mc[1] * mc[2]), hi1(lo1.size());
  for (int i = 0; i < n0; ++i)
    for (int c1 = 0; c1 < mc[1]; ++c1) {
      int a0, a1;
      win(1, c1, a0, a1);
      for (int c2 = 0; c2 < mc[2]; ++c2) {
        float mn = INFINITY, mx = -INFINITY;
        for (int jj = a0; jj <= a1; ++jj) {
          const size_t q = ((size_t)i * n1 + jj) * mc[2] + c2;
          mn = std::fmin(mn, lo2[q]);
          mx = std::fmax(mx, hi2[q]);
        }
        lo1[((size_t)i * mc[1] + c1) * mc[2] + c2] = mn;
        hi1[((size_t)i * mc[1] + c1) * mc[2] + c2] = mx;
      }
    }
  for (int c0 = 0; c0 < mc[0]; ++c0) {
    int a0, a1;
    win(0, c0, a0, a1);
    for (int c12 = 0; c12 < mc[1] * mc[2]; ++c12) {
      float mn = INFINITY, mx = -INFINITY;
      for (int i = a0; i <= a1; ++i) {
        mn = std::fmin(mn, lo1[(size_t)i * mc[1] * mc[2] + c12]);
        mx = std::fmax(mx, hi1[(size_t)i * mc[1] * mc[2] + c12]);
      }
      out.push_back(make_float2(mn, mx));
    }
  }
}

template <class Tp>
static mfa_status upload(Tp** dst, const void* src, size_t bytes, mfa_model m, const char* what) {
  hipError_t e = hipMalloc((void**)dst, bytes ? bytes : 16);
  if (e != hipSuccess) return hip_fail(e, what);
  m->device_bytes += (int64_t)(bytes ? bytes : 16);
  if (bytes) {
    e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  return MFA_OK;
}

extern "C" mfa_status mfa_model_create(const mfa_domain_desc* dom, const mfa_block_desc* blocks,
                                       int32_t nblocks, mfa_dtype storage, mfa_model* out) {
  if (!dom || !blocks || !out) return fail(MFA_E_ARG, "null argument");
  *out = nullptr;
  if (storage != MFA_F32 && storage != MFA_BF16 && storage != MFA_F16)
    return fail(MFA_E_ARG, "storage must be MFA_F32, MFA_BF16 or MFA_F16");
  int64_t nb = 1;
  for (int a = 0; a < 3; ++a) {
    if (dom->grid[a] < 1 || dom->grid[a] > 4096) return fail(MFA_E_ARG, "grid[%d] out of range", a);
    if (!is_fin(dom->lo[a]) || !is_fin(dom->hi[a]) || !(dom->lo[a] < dom->hi[a]))
      return fail(MFA_E_ARG, "domain lo/hi invalid on axis %d", a);
    nb *= dom->grid[a];
  }
  if (!(dom->voxel > 0.0) || !is_fin(dom->voxel)) return fail(MFA_E_ARG, "voxel must be > 0");
  if (nblocks != nb) return fail(MFA_E_ARG, "nblocks %d != grid product %lld", nblocks, (long long)nb);
  if (nb > (1 << 20)) return fail(MFA_E_UNSUPPORTED, "too many blocks");

  // edges
  std::vector<double> edges[3];
  for (int a = 0; a < 3; ++a) {
    const int G = dom->grid[a];
    edges[a].resize(G + 1);
    if (dom->edges[a]) {
      for (int i = 0; i <= G; ++i) edges[a][i] = dom->edges[a][i];
      if (edges[a][0] != dom->lo[a] || edges[a][G] != dom->hi[a])
        return fail(MFA_E_ARG, "edges[%d] must start at lo and end at hi", a);
      for (int i = 0; i < G; ++i)
        if (!(edges[a][i] < edges[a][i + 1]) || !is_fin(edges[a][i + 1]))
          return fail(MFA_E_ARG, "edges[%d] must increase strictly", a);
    } else {
      for (int i = 0; i <= G; ++i)
        edges[a][i] = dom->lo[a] + (dom->hi[a] - dom->lo[a]) * ((double)i / (double)G);
      edges[a][0] = dom->lo[a];
      edges[a][G] = dom->hi[a];
    }
  }

  const int p = blocks[0].degree[0];
  if (p < 1 || p > kMaxDegree) return fail(MFA_E_UNSUPPORTED, "degree %d not in 1..%d", p, kMaxDegree);
  if (p > 5) return fail(MFA_E_UNSUPPORTED, "degree %d: kernels are built for degrees 1..5", p);
  for (int64_t b = 0; b < nb; ++b) {
    const mfa_block_desc& B = blocks[b];
    for (int a = 0; a < 3; ++a) {
      if (B.degree[a] != p)
        return fail(MFA_E_UNSUPPORTED, "block %lld axis %d: all axes and blocks must share degree %d",
                    (long long)b, a, p);
      if (B.n_ctrl[a] < p + 1 || B.n_ctrl[a] > (1 << 16))
        return fail(MFA_E_ARG, "block %lld axis %d: n_ctrl %d not in [p+1, 65536]", (long long)b, a,
                    B.n_ctrl[a]);
    }
    if (!B.ctrl) return fail(MFA_E_ARG, "block %lld: ctrl is null", (long long)b);
    if (B.ctrl_dtype != MFA_F64 && B.ctrl_dtype != MFA_F32)
      return fail(MFA_E_ARG, "block %lld: ctrl_dtype must be MFA_F64 or MFA_F32", (long long)b);
  }

  int current = 0;
  hipError_t he = hipGetDevice(&current);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");

  mfa_model m = new mfa_model_s();
  m->device = current;
  m->degree = p;
  m->storage = storage;
  m->nblocks = (int)nb;
  m->voxel = dom->voxel;
  for (int a = 0; a < 3; ++a) m->grid[a] = dom->grid[a];

  const int es = elem_size(storage);
  std::vector<DevBlock> dblk(nb);
  std::vector<SpanRec> recs;
  std::vector<int32_t> gtab, gmeta(6 * nb, 0);
  std::vector<float> mats;
  std::map<std::vector<float>, int> mat_ids;
  const std::vector<float> canon = uniform_table(p);
  int64_t off = 0;
  m->n.resize(3 * nb);
  m->coff.resize(nb);
  m->rs1.resize(nb);
  for (int64_t b = 0; b < nb; ++b) {
    const mfa_block_desc& B = blocks[b];
    const int b0 = (int)(b / ((int64_t)dom->grid[1] * dom->grid[2]));
    const int b1 = (int)((b / dom->grid[2]) % dom->grid[1]);
    const int b2 = (int)(b % dom->grid[2]);
    const int bi[3] = {b0, b1, b2};
    DevBlock& D = dblk[b];
    for (int a = 0; a < 3; ++a) {
      D.lo[a] = edges[a][bi[a]];
      D.ext[a] = edges[a][bi[a] + 1] - edges[a][bi[a]];
      D.inv_ext[a] = 1.0 / D.ext[a];
      D.n[a] = B.n_ctrl[a];
      D.nsp[a] = B.n_ctrl[a] - p;
      m->n[3 * b + a] = B.n_ctrl[a];
    }
    D.rs1 = (es == 2) ? (B.n_ctrl[2] + (B.n_ctrl[2] & 1)) : B.n_ctrl[2];

    D.ctrl_off = off;
    m->coff[b] = off;
    m->rs1[b] = D.rs1;
    off += (int64_t)B.n_ctrl[0] * B.n_ctrl[1] * D.rs1;
    m->n_ctrl_total += (int64_t)B.n_ctrl[0] * B.n_ctrl[1] * B.n_ctrl[2];
    for (int a = 0; a < 3; ++a) {
      const int n = B.n_ctrl[a];
      std::vector<double> T(n + p + 1);
      if (B.knots[a]) {
        std::memcpy(T.data(), B.knots[a], sizeof(double) * (n + p + 1));
        mfa_status st = check_knots(T.data(), n, p, (int)b, a);
        if (st != MFA_OK) { free_model(m); return st; }
      } else {
        default_knots(n, p, T.data());
      }
      D.rec_off[a] = (int32_t)recs.size();
      for (int j = 0; j < n - p; ++j) {
        const int s = p + j;
        SpanRec r;
        r.t = T[s];
        r.t_next = T[s + 1];
        r.inv_h = (r.t_next > r.t) ? 1.0 / (r.t_next - r.t) : 0.0;
        r.dscale = (float)(r.inv_h * D.inv_ext[a]);
        std::vector<float> tab = (r.t_next > r.t) ? span_table(T.data(), p, s)
                                                  : std::vector<float>(mat_stride(p), 0.f);
        if (near_table(tab, canon)) tab = canon;
        auto it = mat_ids.find(tab);
        if (it == mat_ids.end()) {
          const int id = (int)mat_ids.size();
          mat_ids.emplace(tab, id);
          mats.insert(mats.end(), tab.begin(), tab.end());
          r.mat = id;
        } else {
          r.mat = it->second;
        }
        recs.push_back(r);
      }
      // Span guess table of a non-uniform axis: bins of width at most half
      // the shortest span hold at most one knot each, so the span of the
      // bin's left edge is the exact span or the one before it.
      const int nsp = n - p;
      bool uniform = true;
      double hmin = INFINITY;
      for (int j = 0; j < nsp; ++j) {
        uniform &= T[p + j] == (double)j / (double)nsp;
        if (T[p + j + 1] > T[p + j]) hmin = std::fmin(hmin, T[p + j + 1] - T[p + j]);
      }
      gmeta[6 * b + a] = -1;
      if (!uniform) {
        const int64_t G = std::min<int64_t>(std::max<int64_t>((int64_t)std::ceil(2.0 / hmin), nsp),
                                            std::min<int64_t>(64ll * nsp, 1ll << 20));
        gmeta[6 * b + a] = (int32_t)gtab.size();
        gmeta[6 * b + 3 + a] = (int32_t)G;
        for (int64_t g = 0; g < G; ++g) {
          const double u = (double)g / (double)G;
          const int s = (int)(std::upper_bound(T.data() + p, T.data() + n, u) - T.data()) - 1;
          gtab.push_back(std::min(std::max(s, p), n - 1) - p);
        }
      }
    }
  }
  if (gtab.size() > (size_t)INT32_MAX) { free_model(m); return fail(MFA_E_UNSUPPORTED, "span tables too large"); }
  m->nonuniform = !gtab.empty();
  if (recs.size() > (size_t)INT32_MAX) { free_model(m); return fail(MFA_E_UNSUPPORTED, "too many spans"); }
  // Finest macro cells whose bounds (4 bytes each) take no more memory than
  // the larger of the stored control points and 16 MiB.
  int mc_shift = kMaxMacroShift;
  for (int sh = 0; sh <= kMaxMacroShift; ++sh) {
    int64_t cells = 0;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t c = 1;
      for (int a = 0; a < 3; ++a) c *= (dblk[b].nsp[a] + (1 << sh) - 1) >> sh;
      cells += c;
    }
    if (cells * 4 <= std::max<int64_t>(off * es, 16ll << 20)) {
      mc_shift = sh;
      break;
    }
  }
  const int sc_shift[2] = {mc_shift + kSuperShift[0], mc_shift + kSuperShift[1]};
  for (int64_t b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      dblk[b].mc[a] = (dblk[b].nsp[a] + (1 << mc_shift) - 1) >> mc_shift;
      for (int l = 0; l < 2; ++l)
        dblk[b].sc[l][a] = (dblk[b].nsp[a] + (1 << sc_shift[l]) - 1) >> sc_shift[l];
    }
  // sort tiles of 2^sort_shift spans per axis: the largest whose control-
  // point windows (the tile's spans plus p per axis) hold at most kWinMax
  // values, so the decode stages them in LDS; larger while the model would
  // have more than kMaxBuckets buckets (blocks count at least one bucket
  // each; their windows are then decoded from global memory)
  auto tiles_of = [&](int64_t b, int sh, int a) { return (dblk[b].nsp[a] + (1 << sh) - 1) >> sh; };
  auto count_buckets = [&](int sh) {
    int64_t c = 0;
    for (int64_t b = 0; b < nb; ++b) c += (int64_t)tiles_of(b, sh, 0) * tiles_of(b, sh, 1) * tiles_of(b, sh, 2);
    return c;
  };
  auto max_window = [&](int sh) {
    int64_t w = 0;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t v = 1;
      for (int a = 0; a < 3; ++a) v *= std::min(1 << sh, (int)dblk[b].nsp[a]) + p;
      w = std::max(w, v);
    }
    return w;
  };
  int sort_shift = 0;
  while (sort_shift < 16 && max_window(sort_shift + 1) <= kWinMax) ++sort_shift;
  while (sort_shift < 16 && count_buckets(sort_shift) > kMaxBuckets) ++sort_shift;
  const int64_t buckets = count_buckets(sort_shift);   // > kMaxBuckets: sorted decode rejected
  for (int64_t b = 0, acc = 0; b < nb; ++b) {
    dblk[b].tile_off = (int32_t)acc;
    acc += (int64_t)tiles_of(b, sort_shift, 0) * tiles_of(b, sort_shift, 1) * tiles_of(b, sort_shift, 2);
  }
  m->n_buckets = buckets;
  // control-point window of each sort bucket, in bucket order: the tile's
  // spans plus p control points per axis
  std::vector<BucketWin> bwin;
  if (buckets <= kMaxBuckets) {
    bwin.reserve((size_t)buckets);
    for (int64_t b = 0; b < nb; ++b) {
      int td[3];
      for (int a = 0; a < 3; ++a) td[a] = tiles_of(b, sort_shift, a);
      for (int t0 = 0; t0 < td[0]; ++t0)
        for (int t1 = 0; t1 < td[1]; ++t1)
          for (int t2 = 0; t2 < td[2]; ++t2) {
            const int t[3] = {t0, t1, t2};
            BucketWin w{};
            w.block = (int32_t)b;
            for (int a = 0; a < 3; ++a) {
              const int j0 = t[a] << sort_shift;
              const int j1 = std::min((t[a] + 1) << sort_shift, dblk[b].nsp[a]);   // one past
              w.o[a] = j0;
              w.w[a] = j1 - j0 + p;
            }
            bwin.push_back(w);
          }
    }
  }
  // per block, the data of the sort-bucket computation
  std::vector<SortBlk> sblk((size_t)nb);
  for (int64_t b = 0; b < nb; ++b) {
    for (int a = 0; a < 3; ++a) {
      sblk[b].lo[a] = (float)dblk[b].lo[a];
      // the power-of-two factor is exact, so floor((x - lo) * tscale) is the
      // FP32 span floor((x - lo) * scale) shifted right by sort_shift
      sblk[b].tscale[a] = std::ldexp((float)(dblk[b].inv_ext[a] * (double)dblk[b].nsp[a]), -sort_shift);
      sblk[b].nt[a] = tiles_of(b, sort_shift, a);
    }
    sblk[b].tile_off = dblk[b].tile_off;
  }
  int32_t win_max = 0;
  for (const BucketWin& w : bwin) win_max = std::max(win_max, w.w[0] * w.w[1] * w.w[2]);
  const int64_t pool_bytes = off * es + 64;       // tail pad: 16-bit rows read one word ahead
  if (pool_bytes > 0xFFFFFFFFll) {
    free_model(m);
    return fail(MFA_E_UNSUPPORTED, "stored control points exceed 4 GiB per model");
  }

  // storage rounding
  std::vector<uint8_t> pool((size_t)pool_bytes, 0);
  float vmin = INFINITY, vmax = -INFINITY;
  std::vector<float2> mcb, scb[2];
  for (int64_t b = 0; b < nb; ++b) {
    const mfa_block_desc& B = blocks[b];
    const int n0 = B.n_ctrl[0], n1 = B.n_ctrl[1], n2 = B.n_ctrl[2];
    std::vector<float> V((size_t)n0 * n1 * n2);
    for (int64_t i = 0; i < (int64_t)n0 * n1; ++i) {
      for (int k = 0; k < n2; ++k) {
        const int64_t src = i * n2 + k;
        const double v64 = B.ctrl_dtype == MFA_F64 ? ((const double*)B.ctrl)[src]
                                                   : (double)((const float*)B.ctrl)[src];
        if (!is_fin(v64)) {
          free_model(m);
          return fail(MFA_E_ARG, "block %lld: control point %lld not finite", (long long)b,
                      (long long)src);
        }
        const float v32 = (float)v64;
        const int64_t dst = dblk[b].ctrl_off + i * dblk[b].rs1 + k;
        float stored = v32;
        if (storage == MFA_F32) {
          std::memcpy(&pool[dst * 4], &v32, 4);
        } else if (storage == MFA_BF16) {
          const uint16_t h = to_bf16(v32);
          std::memcpy(&pool[dst * 2], &h, 2);
          stored = bf16_value(h);
        } else {
          const uint16_t h = to_f16(v32);
          if ((h & 0x7C00u) == 0x7C00u) {
            free_model(m);
            return fail(MFA_E_ARG, "block %lld: control point %g overflows FP16", (long long)b, v64);
          }
          std::memcpy(&pool[dst * 2], &h, 2);
          stored = f16_value(h);
        }
        vmin = std::fmin(vmin, stored);
        vmax = std::fmax(vmax, stored);
        V[(size_t)src] = stored;
      }
    }
    dblk[b].mc_off = (int32_t)mcb.size();
    macro_bounds(V, B.n_ctrl, p, mc_shift, dblk[b].mc, mcb);
    for (int l = 0; l < 2; ++l) {
      dblk[b].sc_off[l] = (int32_t)scb[l].size();
      macro_bounds(V, B.n_ctrl, p, sc_shift[l], dblk[b].sc[l], scb[l]);
    }
  }
  m->vmin = vmin;
  m->vmax = vmax;
  // Widen the bounds by a margin above the FP32 evaluation error (basis
  // tables and sums in FP32 stay within ~1e-6 of the exact convex
  // combination relative to max |P|).
  const float margin = 1e-4f * std::fmax(std::fabs(vmin), std::fabs(vmax));
  auto pack16 = [margin](const std::vector<float2>& v) {
    std::vector<uint32_t> o(v.size());
    for (size_t q = 0; q < v.size(); ++q)
      o[q] = (uint32_t)f16_directed(v[q].x - margin, false) |
             ((uint32_t)f16_directed(v[q].y + margin, true) << 16);
    return o;
  };
  const std::vector<uint32_t> mcb16 = pack16(mcb), scb16[2] = {pack16(scb[0]), pack16(scb[1])};
  // the uniform interior table, evaluated from literals by the kernels
  const auto ic = mat_ids.find(canon);
  const int imat = ic == mat_ids.end() ? -1 : ic->second;

  std::vector<double> edge_pool;
  for (int a = 0; a < 3; ++a) m->edges[a] = edges[a];
  int edge_off[3];
  for (int a = 0; a < 3; ++a) {
    edge_off[a] = (int)edge_pool.size();
    edge_pool.insert(edge_pool.end(), edges[a].begin(), edges[a].end());
  }

  std::vector<float> sedges(edge_pool.begin(), edge_pool.end());   // FP32 copy for the sort

  mfa_status st;
  if ((st = upload(&m->d_ctrl, pool.data(), pool.size(), m, "ctrl upload")) != MFA_OK ||
      (st = upload(&m->d_rec, recs.data(), recs.size() * sizeof(SpanRec), m, "span upload")) != MFA_OK ||
      (st = upload(&m->d_mats, mats.data(), mats.size() * sizeof(float), m, "basis upload")) != MFA_OK ||
      (st = upload(&m->d_blocks, dblk.data(), dblk.size() * sizeof(DevBlock), m, "block upload")) != MFA_OK ||
      (st = upload(&m->d_edges, edge_pool.data(), edge_pool.size() * sizeof(double), m, "edge upload")) != MFA_OK ||
      (st = upload(&m->d_mcb, mcb16.data(), mcb16.size() * sizeof(uint32_t), m, "bounds upload")) != MFA_OK ||
      (st = upload(&m->d_scb[0], scb16[0].data(), scb16[0].size() * 4, m, "bounds upload")) != MFA_OK ||
      (st = upload(&m->d_scb[1], scb16[1].data(), scb16[1].size() * 4, m, "bounds upload")) != MFA_OK ||
      (!bwin.empty() &&
       (st = upload(&m->d_bwin, bwin.data(), bwin.size() * sizeof(BucketWin), m, "window upload")) != MFA_OK) ||
      (st = upload(&m->d_sblk, sblk.data(), sblk.size() * sizeof(SortBlk), m, "sort table upload")) != MFA_OK ||
      (st = upload(&m->d_sedges, sedges.data(), sedges.size() * sizeof(float), m, "sort edge upload")) != MFA_OK ||
      (!gtab.empty() &&
       ((st = upload(&m->d_gtab, gtab.data(), gtab.size() * sizeof(int32_t), m, "span table upload")) != MFA_OK ||
        (st = upload(&m->d_gmeta, gmeta.data(), gmeta.size() * sizeof(int32_t), m, "span table upload")) != MFA_OK))) {
    free_model(m);
    return st;
  }
  m->ctrl_bytes = pool_bytes;

  DevModel& dm = m->dm;
  dm.ctrl = m->d_ctrl;
  dm.rec = m->d_rec;
  dm.mats = m->d_mats;
  dm.blocks = m->d_blocks;
  dm.edges = m->d_edges;
  dm.ctrl_bytes = pool_bytes;
  for (int a = 0; a < 3; ++a) {
    dm.edge_off[a] = edge_off[a];
    dm.grid[a] = dom->grid[a];
    dm.box_lo[a] = dom->lo[a];
    dm.box_hi[a] = dom->hi[a];
    dm.edge_scale[a] = (double)dom->grid[a] / (dom->hi[a] - dom->lo[a]);
  }
  dm.nblocks = (int)nb;
  dm.mat_stride = mat_stride(p);
  dm.n_mats = (int)mat_ids.size();
  dm.n_rec = (int)recs.size();
  dm.imat = imat;
  dm.mc_shift = mc_shift;
  dm.sort_shift = sort_shift;
  dm.mcb = m->d_mcb;
  for (int l = 0; l < 2; ++l) {
    dm.scb[l] = m->d_scb[l];
    dm.sc_shift[l] = sc_shift[l];
  }
  dm.bwin = m->d_bwin;
  dm.sblk = m->d_sblk;
  dm.sedges = m->d_sedges;
  dm.n_edges = (int32_t)edge_pool.size();
  dm.gtab = m->d_gtab;
  dm.gmeta = m->d_gmeta;
  dm.win_max = win_max;
  dm.b0 = dblk[0];
  *out = m;
  return MFA_OK;
}

extern "C" mfa_status mfa_model_destroy(mfa_model m) {
  free_model(m);
  return MFA_OK;
}

extern "C" mfa_status mfa_model_info(mfa_model m, mfa_model_info_t* info) {
  if (!m || !info) return fail(MFA_E_ARG, "null argument");
  info->device_bytes = m->device_bytes;
  info->ctrl_bytes = m->ctrl_bytes;
  info->n_ctrl_total = m->n_ctrl_total;
  info->nblocks = m->nblocks;
  info->degree = m->degree;
  info->storage = m->storage;
  info->vmin = m->vmin;
  info->vmax = m->vmax;
  info->voxel = m->voxel;
  info->device = m->device;
  return MFA_OK;
}

mfa_status check_device(mfa_model m) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != m->device)
    return fail(MFA_E_ARG, "current device %d is not the model's device %d", cur, m->device);
  return MFA_OK;
}

extern "C" mfa_status mfa_model_export_ctrl(mfa_model m, int32_t block, void* dst, int64_t dst_bytes) {
  if (!m || !dst) return fail(MFA_E_ARG, "null argument");
  if (block < 0 || block >= m->nblocks) return fail(MFA_E_ARG, "block %d out of range", block);
  const int es = elem_size(m->storage);
  const int n0 = m->n[3 * block], n1 = m->n[3 * block + 1], n2 = m->n[3 * block + 2];
  const int64_t need = (int64_t)n0 * n1 * n2 * es;
  if (dst_bytes < need) return fail(MFA_E_ARG, "dst_bytes %lld < %lld", (long long)dst_bytes, (long long)need);
  mfa_status st = check_device(m);
  if (st != MFA_OK) return st;
  const int rs = m->rs1[block];
  std::vector<uint8_t> tmp((size_t)n0 * n1 * rs * es);
  hipError_t e = hipMemcpy(tmp.data(), (const uint8_t*)m->d_ctrl + m->coff[block] * es, tmp.size(),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "export copy");
  for (int64_t i = 0; i < (int64_t)n0 * n1; ++i)
    std::memcpy((uint8_t*)dst + i * n2 * es, tmp.data() + i * rs * es, (size_t)n2 * es);
  return MFA_OK;
}

// ------------------------------------------------------------------ decode
Storage storage_of(mfa_model m) {
  return m->storage == MFA_F32 ? Storage::F32 : m->storage == MFA_BF16 ? Storage::BF16 : Storage::F16;
}

// Arguments shared by the point decodes.
static mfa_status check_points(mfa_model m, const float* xyz, int64_t n, uint32_t flags,
                               const float* out) {
  if (!m) return fail(MFA_E_ARG, "null model");
  if (n < 0 || n >= (1ll << 31)) return fail(MFA_E_ARG, "n = %lld out of range", (long long)n);
  if (flags & ~(MFA_DECODE_SORTED | MFA_DECODE_VALUE)) return fail(MFA_E_ARG, "unknown flags 0x%x", flags);
  if (n > 0 && (!xyz || !out)) return fail(MFA_E_ARG, "null xyz/out");
  return MFA_OK;
}

// Scratch of a sorted decode of n points over nb buckets, one region after
// another (256-byte aligned): one 16-byte record per point, counts, starts
// and cursors per bucket, the decode items and their count, and with the
// two-level split the coarse cursors, a second record per point and each
// point's position in the coarse order.
struct SortLayout {
  size_t o_hist, o_start, o_cur, o_items, o_nitems, o_ccur, o_tmp, o_tpos, bytes;
  bool two;
  int fine_shift;
};

static SortLayout sort_layout(int64_t n, int64_t nb) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  SortLayout L{};
  const size_t nbk = (size_t)nb;
  const size_t n_items = (size_t)((n + kTilePoints - 1) / kTilePoints) + nbk;
  L.o_hist = al(16 * (size_t)n);
  L.o_start = L.o_hist + al(4 * nbk);
  L.o_cur = L.o_start + al(4 * (nbk + 1));
  L.o_items = L.o_cur + al(4 * nbk);
  L.o_nitems = L.o_items + al(8 * n_items);
  L.o_ccur = L.o_nitems + al(4);
  L.two = nbk > (size_t)kOneLevelBuckets;
  L.fine_shift = 0;
  while ((nb + (1ll << L.fine_shift) - 1) >> L.fine_shift > kCoarseBuckets) ++L.fine_shift;
  L.o_tmp = L.o_ccur + al(4 * kCoarseBuckets * kCursorStride);
  L.o_tpos = L.o_tmp + al(16 * (size_t)n);
  L.bytes = L.two ? L.o_tpos + al(4 * (size_t)n) : L.o_ccur;
  return L;
}

// Sorts and decodes with the scratch at w (device, >= sort_layout().bytes).
static mfa_status sorted_decode(mfa_model m, uint8_t* w, const SortLayout& L, const float* xyz,
                                int64_t n, bool grad, float* out, int32_t* dbg, void* stream) {
  SortArgs sa{};
  sa.xyz = xyz;
  sa.n = n;
  sa.rec = (float4*)w;
  sa.hist = (uint32_t*)(w + L.o_hist);
  sa.start = (uint32_t*)(w + L.o_start);
  sa.cursor = (uint32_t*)(w + L.o_cur);
  sa.items = (int2*)(w + L.o_items);
  sa.n_items = (int32_t*)(w + L.o_nitems);
  sa.nb = (int32_t)m->n_buckets;
  sa.fine_shift = L.fine_shift;
  sa.tmp = L.two ? (float4*)(w + L.o_tmp) : nullptr;
  sa.ccursor = L.two ? (uint32_t*)(w + L.o_ccur) : nullptr;
  // two levels: the results go through the coarse order (writes within one
  // coarse key's region at a time rather than over the whole output), except
  // with debug outputs, which are written at the input positions directly
  sa.tpos = L.two && !dbg ? (uint32_t*)(w + L.o_tpos) : nullptr;
  sa.bkt = sa.tpos ? (uint16_t*)w : nullptr;         // in the region of rec (filled last)
  hipError_t e = launch_decode_sorted(m->dm, m->degree, storage_of(m), kernel_kind(m), grad, sa, out,
                                      dbg, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "sorted decode launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_decode_points(mfa_model m, const float* xyz, int64_t n, uint32_t flags,
                                        float* out, int32_t* dbg, void* stream) {
  mfa_status st = check_points(m, xyz, n, flags, out);
  if (st != MFA_OK || n == 0) return st;
  st = check_device(m);
  if (st != MFA_OK) return st;
  const bool grad = !(flags & MFA_DECODE_VALUE);
  if (flags & MFA_DECODE_SORTED) {
    if (m->n_buckets > kMaxBuckets)
      return fail(MFA_E_UNSUPPORTED, "sorted decode supports at most %d buckets (blocks)", kMaxBuckets);
    const SortLayout L = sort_layout(n, m->n_buckets);
    // The scratch is the model's: a sorted call waits for the previous
    // sorted call's kernels (an event recorded after them) before it reuses
    // or replaces the buffer, so calls on different streams are ordered
    // rather than racing.
    std::lock_guard<std::mutex> guard(m->ws_mu);
    hipError_t e;
    if (!m->ws_done) {
      e = hipEventCreateWithFlags(&m->ws_done, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "scratch event");
    }
    if (L.bytes > m->ws_bytes) {
      if (m->d_ws) {
        e = hipEventSynchronize(m->ws_done);     // the previous sorted call's kernels
        if (e != hipSuccess) return hip_fail(e, "scratch wait");
        e = hipFree(m->d_ws);
        m->d_ws = nullptr;
        m->device_bytes -= (int64_t)m->ws_bytes;
        m->ws_bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "scratch free");
      }
      e = hipMalloc(&m->d_ws, L.bytes);
      if (e != hipSuccess) {
        m->d_ws = nullptr;
        return fail(MFA_E_NOMEM, "scratch for sorted decode (%zu bytes): %s", L.bytes,
                    hipGetErrorString(e));
      }
      m->ws_bytes = L.bytes;
      m->device_bytes += (int64_t)L.bytes;
    } else if (m->ws_used && (hipStream_t)stream != m->ws_stream) {
      e = hipStreamWaitEvent((hipStream_t)stream, m->ws_done, 0);
      if (e != hipSuccess) return hip_fail(e, "scratch stream wait");
    }
    st = sorted_decode(m, (uint8_t*)m->d_ws, L, xyz, n, grad, out, dbg, stream);
    if (st != MFA_OK) return st;
    e = hipEventRecord(m->ws_done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "scratch event record");
    m->ws_stream = (hipStream_t)stream;
    m->ws_used = true;
    return MFA_OK;
  }
  hipError_t e = launch_decode_points(m->dm, m->degree, storage_of(m), kernel_kind(m), grad, xyz, n,
                                      out, dbg, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_points launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_decode_points_noalloc(mfa_model m, const float* xyz, int64_t n,
                                                uint32_t flags, float* out, int32_t* dbg,
                                                void* stream) {
  mfa_status st = check_points(m, xyz, n, flags, out);
  if (st != MFA_OK) return st;
  if (m->n_buckets > kMaxBuckets)
    return fail(MFA_E_UNSUPPORTED, "sorted decode supports at most %d buckets (blocks)", kMaxBuckets);
  const SortLayout L = sort_layout(n, m->n_buckets);
  if (L.bytes > kStaticScratchBytes) {
    // largest n whose scratch fits, for the message
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (sort_layout(mid, m->n_buckets).bytes <= kStaticScratchBytes) lo = mid; else hi = mid - 1;
    }
    return fail(MFA_E_ARG, "n = %lld needs %zu bytes of scratch, more than the %zu of the static "
                "scratch (at most %lld points for this model)", (long long)n, L.bytes,
                kStaticScratchBytes, (long long)lo);
  }
  if (n == 0) return MFA_OK;
  st = check_device(m);
  if (st != MFA_OK) return st;
  void* w = nullptr;
  hipError_t e = static_scratch(&w);
  if (e != hipSuccess) return hip_fail(e, "static scratch address");
  return sorted_decode(m, (uint8_t*)w, L, xyz, n, !(flags & MFA_DECODE_VALUE), out, dbg, stream);
}

extern "C" mfa_status mfa_decode_grid(mfa_model m, const double* const axis_u[3], const int32_t res[3],
                                      uint32_t flags, float* out, int32_t* spans, void* stream) {
  if (!m || !axis_u || !res || !out) return fail(MFA_E_ARG, "null argument");
  if (flags & ~MFA_DECODE_VALUE) return fail(MFA_E_ARG, "unknown flags 0x%x", flags);
  if (m->nblocks != 1) return fail(MFA_E_ARG, "grid decode needs a single-block model");
  int64_t total = 1;
  for (int a = 0; a < 3; ++a) {
    if (!axis_u[a]) return fail(MFA_E_ARG, "axis_u[%d] is null", a);
    if (res[a] < 1) return fail(MFA_E_ARG, "res[%d] = %d < 1", a, res[a]);
    total *= res[a];
  }
  if (res[1] > 4 * 65535 || res[0] > 64 * 65535) return fail(MFA_E_ARG, "res too large for the launch");
  if (total >= (1ll << 40)) return fail(MFA_E_ARG, "grid too large");
  mfa_status st = check_device(m);
  if (st != MFA_OK) return st;
  GridArgs ga{};
  for (int a = 0; a < 3; ++a) {
    ga.axis[a] = axis_u[a];
    ga.res[a] = res[a];
  }
  ga.out = out;
  ga.spans = spans;
  hipError_t e = launch_decode_grid(m->dm, m->degree, storage_of(m), !(flags & MFA_DECODE_VALUE), ga,
                                    (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_grid launch");
  return MFA_OK;
}

// ------------------------------------------------------------------ render
// Validated kernel arguments of a render; voxel: the default step is half of it.
static mfa_status render_args_core(double voxel, const mfa_camera* cam, const mfa_render_params* rp,
                                   int32_t w, int32_t h, float* rgba, const mfa_render_debug* dbg,
                                   RenderArgs* out, bool need_tf) {
  if (!cam || !rp || !rgba) return fail(MFA_E_ARG, "null argument");
  if (w < 1 || h < 1 || w > 16384 || h > 16384) return fail(MFA_E_ARG, "image %dx%d out of range", w, h);
  if (cam->kind != MFA_ORTHO && cam->kind != MFA_PERSPECTIVE) return fail(MFA_E_ARG, "camera kind");
  for (int a = 0; a < 3; ++a)
    if (!is_fin(cam->eye[a]) || !is_fin(cam->forward[a]) || !is_fin(cam->right[a]) || !is_fin(cam->up[a]))
      return fail(MFA_E_ARG, "camera vectors must be finite");
  if (!is_fin(cam->sx) || !is_fin(cam->sy)) return fail(MFA_E_ARG, "camera scales must be finite");
  if (need_tf && !rp->tf_rgba) return fail(MFA_E_ARG, "tf_rgba is null");
  if (need_tf && (!(rp->vmin < rp->vmax) || !std::isfinite(rp->vmin) || !std::isfinite(rp->vmax)))
    return fail(MFA_E_ARG, "need finite vmin < vmax");
  const double step = rp->step == 0.0 ? 0.5 * voxel : rp->step;
  if (!(step > 0.0) || !is_fin(step)) return fail(MFA_E_ARG, "step must be > 0");
  if (rp->max_samples < 1) return fail(MFA_E_ARG, "max_samples must be >= 1");
  if (!(rp->g0 > 0.f) || !std::isfinite(rp->g0)) return fail(MFA_E_ARG, "g0 must be > 0");
  if (rp->shininess < 0 || rp->shininess > 1024) return fail(MFA_E_ARG, "shininess out of range");
  if (!std::isfinite(rp->ka) || !std::isfinite(rp->kd) || !std::isfinite(rp->ks) ||
      std::isnan(rp->ert_alpha))
    return fail(MFA_E_ARG, "shading parameters must be finite");
  if (dbg && dbg->alpha && dbg->alpha_stride < rp->max_samples)
    return fail(MFA_E_ARG, "alpha_stride %d < max_samples %d", dbg->alpha_stride, rp->max_samples);
  RenderArgs r{};
  r.tf = rp->tf_rgba;
  r.rgba = rgba;
  r.nsamp = dbg ? dbg->nsamp : nullptr;
  r.neval = dbg ? dbg->neval : nullptr;
  r.alpha = dbg ? dbg->alpha : nullptr;
  r.alpha_stride = dbg ? dbg->alpha_stride : 0;
  r.w = w;
  r.h = h;
  r.kind = cam->kind;
  r.max_samples = rp->max_samples;
  r.shininess = rp->shininess;
  r.vmin = rp->vmin;
  r.inv_range = need_tf ? (float)(1.0 / ((double)rp->vmax - (double)rp->vmin)) : 0.f;
  r.ert_alpha = rp->ert_alpha;
  r.ka = rp->ka;
  r.kd = rp->kd;
  r.ks = rp->ks;
  r.g0 = rp->g0;
  for (int a = 0; a < 3; ++a) {
    r.eye[a] = cam->eye[a];
    r.fwd[a] = cam->forward[a];
    r.right[a] = cam->right[a];
    r.up[a] = cam->up[a];
  }
  r.sx = cam->sx;
  r.sy = cam->sy;
  r.step = step;
  r.inv_step = 1.0 / step;
  *out = r;
  return MFA_OK;
}

mfa_status make_render_args(mfa_model m, const mfa_camera* cam, const mfa_render_params* rp,
                            int32_t w, int32_t h, float* rgba, const mfa_render_debug* dbg,
                            RenderArgs* out, bool need_tf) {
  if (!m) return fail(MFA_E_ARG, "null argument");
  return render_args_core(m->voxel, cam, rp, w, h, rgba, dbg, out, need_tf);
}

extern "C" mfa_status mfa_render_volume(const mfa_volume_desc* vol, const mfa_camera* cam,
                                        const mfa_render_params* rp, int32_t w, int32_t h,
                                        float* rgba, const mfa_render_debug* dbg, void* stream) {
  if (!vol) return fail(MFA_E_ARG, "null volume");
  if (vol->kind < MFA_FILTER_TRILINEAR || vol->kind > MFA_FIELD_MARSCHNER_LOBB)
    return fail(MFA_E_ARG, "unknown volume kind %d", vol->kind);
  VolArgs v{};
  double hmin = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (!is_fin(vol->lo[a]) || !is_fin(vol->hi[a]) || !(vol->lo[a] < vol->hi[a]))
      return fail(MFA_E_ARG, "axis %d: need finite lo < hi", a);
    if (vol->dims[a] < 2 || vol->dims[a] > (1 << 16))
      return fail(MFA_E_ARG, "axis %d: %d samples outside [2, 65536]", a, vol->dims[a]);
    v.n[a] = vol->dims[a];
    v.lo[a] = vol->lo[a];
    v.hi[a] = vol->hi[a];
    v.h[a] = (vol->hi[a] - vol->lo[a]) / (double)(vol->dims[a] - 1);
    v.inv_hd[a] = 1.0 / v.h[a];
    v.inv_h[a] = (float)v.inv_hd[a];
    hmin = std::fmin(hmin, v.h[a]);
  }
  if (vol->kind != MFA_FIELD_MARSCHNER_LOBB && !vol->samples)
    return fail(MFA_E_ARG, "null samples");
  v.v = vol->samples;
  v.bytes = 4ll * v.n[0] * v.n[1] * v.n[2];
  RenderArgs r;
  mfa_status st = render_args_core(hmin, cam, rp, w, h, rgba, dbg, &r, true);
  if (st != MFA_OK) return st;
  hipError_t e = launch_volume(v, vol->kind, r, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "volume render launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_render_frame(mfa_model m, const mfa_camera* cam, const mfa_render_params* rp,
                                       int32_t w, int32_t h, float* rgba, const mfa_render_debug* dbg,
                                       void* stream) {
  RenderArgs r;
  mfa_status st = make_render_args(m, cam, rp, w, h, rgba, dbg, &r);
  if (st != MFA_OK) return st;
  st = check_device(m);
  if (st != MFA_OK) return st;
  hipError_t e = launch_render(m->dm, m->degree, storage_of(m), kernel_kind(m), r, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "render launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_render_partial(mfa_model m, const mfa_camera* cam,
                                         const mfa_render_params* rp, const int32_t block_lo[3],
                                         const int32_t block_hi[3], int32_t w, int32_t h,
                                         float* rgba, double* key, const mfa_render_debug* dbg,
                                         void* stream) {
  RenderArgs r;
  mfa_status st = make_render_args(m, cam, rp, w, h, rgba, dbg, &r);
  if (st != MFA_OK) return st;
  if (!block_lo || !block_hi || !key) return fail(MFA_E_ARG, "null block_lo / block_hi / key");
  for (int a = 0; a < 3; ++a)
    if (block_lo[a] < 0 || block_lo[a] >= block_hi[a] || block_hi[a] > m->grid[a])
      return fail(MFA_E_ARG, "axis %d: block range [%d, %d) outside [0, %d) or empty", a,
                  block_lo[a], block_hi[a], m->grid[a]);
  r.partial = 1;
  for (int a = 0; a < 3; ++a) {
    r.reg_lo[a] = block_lo[a];
    r.reg_hi[a] = block_hi[a];
    r.reg_box_lo[a] = m->edges[a][block_lo[a]];
    r.reg_box_hi[a] = m->edges[a][block_hi[a]];
  }
  r.key = key;
  st = check_device(m);
  if (st != MFA_OK) return st;
  hipError_t e = launch_render(m->dm, m->degree, storage_of(m), kernel_kind(m), r, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "partial render launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_render_iso(mfa_model m, const mfa_camera* cam,
                                     const mfa_render_params* rp, float iso, const float rgb[3],
                                     int32_t w, int32_t h, float* rgba, double* depth,
                                     const mfa_render_debug* dbg, void* stream) {
  RenderArgs r;
  mfa_status st = make_render_args(m, cam, rp, w, h, rgba, dbg, &r, false);
  if (st != MFA_OK) return st;
  if (!std::isfinite(iso)) return fail(MFA_E_ARG, "iso must be finite");
  if (!rgb) return fail(MFA_E_ARG, "null rgb");
  for (int c = 0; c < 3; ++c) {
    if (!std::isfinite(rgb[c])) return fail(MFA_E_ARG, "rgb must be finite");
    r.iso_rgb[c] = rgb[c];
  }
  if (dbg && dbg->alpha) return fail(MFA_E_ARG, "the isosurface render has no alpha output");
  r.iso = iso;
  r.key = depth;
  r.tf = nullptr;
  st = check_device(m);
  if (st != MFA_OK) return st;
  hipError_t e = launch_iso(m->dm, m->degree, storage_of(m), kernel_kind(m), r, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "isosurface render launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_composite_over(int32_t g, const float* const* images,
                                         const double* const* keys, int32_t w, int32_t h,
                                         float* out, void* stream) {
  if (g < 1 || g > kMaxPartials) return fail(MFA_E_ARG, "g = %d outside [1, %d]", g, kMaxPartials);
  if (!images || !keys || !out) return fail(MFA_E_ARG, "null images / keys / out");
  if (w < 1 || h < 1 || w > 16384 || h > 16384) return fail(MFA_E_ARG, "image %dx%d out of range", w, h);
  CompositeArgs c{};
  for (int i = 0; i < g; ++i) {
    if (!images[i] || !keys[i]) return fail(MFA_E_ARG, "null image or key %d", i);
    c.images[i] = reinterpret_cast<const float4*>(images[i]);
    c.keys[i] = keys[i];
  }
  c.g = g;
  c.npix = (int64_t)w * h;
  c.out = reinterpret_cast<float4*>(out);
  hipError_t e = launch_composite(c, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "composite launch");
  return MFA_OK;
}

// ------------------------------------------------------------------ host utilities
extern "C" mfa_status mfa_quantize(const double* src, int64_t n, mfa_dtype dtype, void* dst) {
  if (n < 0 || (n > 0 && (!src || !dst))) return fail(MFA_E_ARG, "bad buffers");
  if (dtype != MFA_F32 && dtype != MFA_BF16 && dtype != MFA_F16) return fail(MFA_E_ARG, "dtype");
  for (int64_t i = 0; i < n; ++i) {
    const float v = (float)src[i];
    if (dtype == MFA_F32) ((uint32_t*)dst)[i] = f32_bits(v);
    else if (dtype == MFA_BF16) ((uint16_t*)dst)[i] = to_bf16(v);
    else ((uint16_t*)dst)[i] = to_f16(v);
  }
  return MFA_OK;
}

extern "C" mfa_status mfa_default_knots(int32_t n, int32_t p, double* dst) {
  if (!dst || p < 1 || p > kMaxDegree || n < p + 1) return fail(MFA_E_ARG, "bad n/p");
  default_knots(n, p, dst);
  return MFA_OK;
}

extern "C" const char* mfa_last_error(void) { return g_err.c_str(); }

extern "C" const char* mfa_version(void) { return "mfa-gfx950 0.1"; }
