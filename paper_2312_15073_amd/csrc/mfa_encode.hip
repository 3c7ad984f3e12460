// Fixed-knot least-squares encoding of samples on a tensor grid (paper
// Sec. IV-A2 "MFA Encoding"; the parameterisation and initial fit of Fig. 1,
// before any knot insertion).  The control points P minimise the sum of
// squared differences between the spline and the samples F; with samples on
// a tensor grid the design matrix is the Kronecker product of the per-axis
// collocation matrices B_a[i][j] = N_{j,p}(u_a[i]), whose pseudo-inverse is
// the Kronecker product of the per-axis pseudo-inverses, so
//     P = F x_0 B0+ x_1 B1+ x_2 B2+,   B+ = (B^T B)^-1 B^T.
// The host builds each B_a (exact FP64 span rule, de Boor's triangular
// scheme for the basis values) and B_a+ by a banded Cholesky factorisation
// of the Gram matrix B_a^T B_a (bandwidth p); the device applies the three
// mode products, which are dense contractions, as FP64 GEMMs on the matrix
// cores (v_mfma_f64_16x16x4f64).
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mfa_model.h"

namespace mfa {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// C[b] = A[b] * B[b] for b < batch: element (m, k) of A at A[m * lda + k]
// (A[k * lda + m] when TRANS_A), element (k, n) of B at B[k * ldb + n],
// element (m, n) of C at C[m * ldc + n] (C[n * ldc + m] when c_trans);
// s* are the batch strides in elements.  The
// per-axis tables are stored transposed (N_a x n_a), so that the 16 lanes
// reading one k of a fragment read 16 consecutive values.
struct GemmArgs {
  int64_t M, N, K, batch;
  const double* A;
  int64_t lda, sA;
  const void* B;
  int64_t ldb, sB;
  double* C;
  int64_t ldc, sC;
  int32_t c_trans;     // element (m, n) of C at C[n * ldc + m]
  // split-K (a product with too few tiles to fill the chip): split > 1
  // chunks of kc values of K (a multiple of 4) per tile, each stored plain
  // into part[((chunk * batch + b) * M + m) * N + n] and summed by split_sum_k
  int64_t split, kc;
  double* part;
};

constexpr int kGemmBlock = 256;   // 4 waves, each computing its own C tile
constexpr int kGemmTile = 32;     // C tile rows per wave: 2 MFMA blocks of 16 (columns: NT blocks)

// One wave per 32 x 16 NT tile of C; tiles are numbered with the M tile
// fastest, so the waves of a workgroup share the columns of B they read
// (with ERR below, N fastest: there the waves share rows of A).
// Per step of 4 along K each lane supplies A(m0 + 16t + lane % 16, k) and
// B(k, n0 + 16u + lane % 16) with k = k0 + lane / 16, and the MFMA leaves
// element (i, j) of a 16 x 16 block in lane j + 16 * (i % 4), register
// i / 4.  Lanes past the last row of A or column of B read the last one
// instead (in bounds): they only feed outputs that are not stored, so the
// main loop has no predicates; the K tail runs one step with zeros past K.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;   // global-memory pointer

// With ERR the GEMM is the last product of a reconstruction: instead of
// storing C it takes every element's relative error against the samples,
// |C(m, n) - F(m, n)| * inv_range (F(m, n) at f[m * ldf + n], inv_range
// read from device memory), and stores
// per tile the largest error of each of its rows, rowpart[jn * M + m], and
// of each of its columns, colpart[im * N + n] (jn, im: the tile's column
// and row index); out-of-range elements count as 0.
constexpr int kErrNT = 2;         // the error product's tiles: 32 x 32 (32 x 64 measured slower)

struct ErrOut {
  const float* f;
  int64_t ldf;
  const double* inv_range;
  double* rowpart;
  double* colpart;
};

constexpr int kGemmUnroll = 4;    // K steps whose loads are issued together

template <typename TB, bool TRANS_A, bool ERR, int NT>
__global__ __launch_bounds__(kGemmBlock) void gemm_f64_k(const double* __restrict__ gA,
                                                         const TB* __restrict__ gB,
                                                         double* __restrict__ gC, GemmArgs g,
                                                         ErrOut eo) {
  const int lane = threadIdx.x & 63;
  // Workgroups are dealt to the 8 XCDs in turn (physical block x to XCD
  // x % 8); renumber them so that each XCD runs a contiguous range of
  // logical blocks, whose tiles share operand strips in that XCD's L2.
  const int64_t nb = gridDim.x, xq = nb / 8, xr = nb % 8, xcd = blockIdx.x % 8, xi = blockIdx.x / 8;
  const int64_t lb = xcd < xr ? xcd * (xq + 1) + xi : xr * (xq + 1) + (xcd - xr) * xq + xi;
  const int64_t w = lb * (kGemmBlock / 64) + (threadIdx.x >> 6);
  constexpr int TN = 16 * NT;                          // tile width along N
  const int64_t tm = (g.M + kGemmTile - 1) / kGemmTile, tn = (g.N + TN - 1) / TN;
  const int64_t S = g.split > 1 ? g.split : 1;
  if (w >= tm * tn * g.batch * S) return;              // whole wave
  // tiles numbered with M fastest (the waves of a run share B columns), or
  // N fastest for the error product (few, narrow B columns; tall A)
  const int64_t im = ERR ? (w / tn) % tm : w % tm, jn = ERR ? w % tn : (w / tm) % tn;
  const int64_t b = (w / (tm * tn)) / S, chunk = (w / (tm * tn)) % S;
  const int64_t k_begin = S > 1 ? chunk * g.kc : 0;
  const int64_t K = S > 1 ? min(g.kc, g.K - k_begin) : g.K;
  const int c16 = lane & 15, q = lane >> 4;
  const int64_t m0 = im * kGemmTile, n0 = jn * TN;
  const double* A0 = gA + b * g.sA + (TRANS_A ? k_begin * g.lda : k_begin);
  const TB* B0 = gB + b * g.sB + k_begin * g.ldb;
  gptr<double> pa[2];
  gptr<TB> pb[NT];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t m = min(m0 + 16 * t + c16, g.M - 1);
    pa[t] = (gptr<double>)(TRANS_A ? A0 + (int64_t)q * g.lda + m : A0 + m * g.lda + q);
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int64_t n = min(n0 + 16 * u + c16, g.N - 1);
    pb[u] = (gptr<TB>)(B0 + (int64_t)q * g.ldb + n);
  }
  const int64_t step_a = TRANS_A ? 4 * g.lda : 4, step_b = 4 * g.ldb;
  v4d acc[2][NT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[t][u] = v4d{0.0, 0.0, 0.0, 0.0};
  auto mma = [&](const double (&a)[2], const double (&bv)[NT]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bv[u], acc[t][u], 0, 0, 0);
  };
  // the error product's samples are loaded before the K loop, so that their
  // latency overlaps the products (rows and columns clamped in bounds, the
  // ones past the edge are masked in the epilogue)
  float fv[2][NT][4];
  double inv_range = 0.0;
  if constexpr (ERR) {
    inv_range = *eo.inv_range;
    gptr<float> F = (gptr<float>)eo.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = min(m0 + 16 * t + q + 4 * r, g.M - 1), n = min(n0 + 16 * u + c16, g.N - 1);
          fv[t][u][r] = F[m * eo.ldf + n];
        }
  }
  const int64_t kfull = K & ~(int64_t)3;
  int64_t k0 = 0;
  for (; k0 + 4 * kGemmUnroll <= kfull; k0 += 4 * kGemmUnroll) {
    double a[kGemmUnroll][2];
    TB bt[kGemmUnroll][NT];
#pragma unroll
    for (int s = 0; s < kGemmUnroll; ++s) {
#pragma unroll
      for (int t = 0; t < 2; ++t) a[s][t] = pa[t][s * step_a];
#pragma unroll
      for (int u = 0; u < NT; ++u) bt[s][u] = pb[u][s * step_b];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) pa[t] += kGemmUnroll * step_a;
#pragma unroll
    for (int u = 0; u < NT; ++u) pb[u] += kGemmUnroll * step_b;
#pragma unroll
    for (int s = 0; s < kGemmUnroll; ++s) {
      double bv[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) bv[u] = (double)bt[s][u];
      mma(a[s], bv);
    }
  }
  for (; k0 < kfull; k0 += 4) {
    double a[2], bv[NT];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = *pa[t];
      pa[t] += step_a;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      bv[u] = (double)*pb[u];
      pb[u] += step_b;
    }
    mma(a, bv);
  }
  if (kfull < K) {
    const bool kin = kfull + q < K;
    double a[2], bv[NT];
#pragma unroll
    for (int t = 0; t < 2; ++t) a[t] = kin ? *pa[t] : 0.0;
#pragma unroll
    for (int u = 0; u < NT; ++u) bv[u] = kin ? (double)*pb[u] : 0.0;
    mma(a, bv);
  }
  if constexpr (ERR) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + 16 * t + q + 4 * r, n = n0 + 16 * u + c16;
          acc[t][u][r] = (m < g.M && n < g.N)
                             ? fabs(acc[t][u][r] - (double)fv[t][u][r]) * inv_range
                             : 0.0;
        }
    // rows: the 16 lanes of one q hold a row's 16 NT columns (NT per lane)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = acc[t][0][r];
#pragma unroll
        for (int u = 1; u < NT; ++u) v = fmax(v, acc[t][u][r]);
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) v = fmax(v, __shfl_xor(v, o));
        const int64_t m = m0 + 16 * t + q + 4 * r;
        if (c16 == 0 && m < g.M) eo.rowpart[jn * g.M + m] = v;
      }
    // columns: a lane holds 8 rows of a column, the four q groups the rest
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) v = fmax(v, acc[t][u][r]);
      v = fmax(v, __shfl_xor(v, 16));
      v = fmax(v, __shfl_xor(v, 32));
      const int64_t n = n0 + 16 * u + c16;
      if (q == 0 && n < g.N) eo.colpart[im * g.N + n] = v;
    }
  } else {
    double* __restrict__ C = gC + b * g.sC;
    double* __restrict__ Pc = S > 1 ? g.part + (chunk * g.batch + b) * g.M * g.N : nullptr;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + 16 * t + q + 4 * r, n = n0 + 16 * u + c16;
          if (m < g.M && n < g.N) {
            if (S > 1)
              Pc[m * g.N + n] = acc[t][u][r];
            else
              C[g.c_trans ? n * g.ldc + m : m * g.ldc + n] = acc[t][u][r];
          }
        }
  }
}

// C = sum over the split chunks of part (see GemmArgs): one thread per
// element of C, in C's own layout.
__global__ __launch_bounds__(256) void split_sum_k(GemmArgs g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = g.M * g.N;
  if (i >= g.batch * per) return;
  const int64_t b = i / per, m = (i % per) / g.N, n = i % g.N;
  double v = 0.0;
  for (int64_t c = 0; c < g.split; ++c) v += g.part[(c * g.batch + b) * per + m * g.N + n];
  g.C[b * g.sC + (g.c_trans ? n * g.ldc + m : m * g.ldc + n)] = v;
}

template <typename TB, bool TRANS_A, bool ERR = false, int NT = 2>
hipError_t gemm(const GemmArgs& g, hipStream_t st, const ErrOut& eo = ErrOut{}) {
  const int64_t S = g.split > 1 ? g.split : 1;
  const int64_t tiles = ((g.M + kGemmTile - 1) / kGemmTile) * ((g.N + 16 * NT - 1) / (16 * NT)) *
                        g.batch * S;
  const int64_t blocks = (tiles + kGemmBlock / 64 - 1) / (kGemmBlock / 64);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (ERR && (g.batch != 1 || S > 1)) return hipErrorInvalidValue;
  if (S > 1 && (!g.part || g.kc < 4 || g.kc % 4 != 0 || (S - 1) * g.kc >= g.K))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_f64_k<TB, TRANS_A, ERR, NT>), dim3((unsigned)blocks), dim3(kGemmBlock), 0, st,
                     g.A, static_cast<const TB*>(g.B), g.C, g, eo);
  if (S > 1) {
    const int64_t n = g.batch * g.M * g.N;
    hipLaunchKernelGGL(split_sum_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

// Split-K for a product with few tiles (fewer waves than the chip holds
// twice over): up to 8 chunks of at least 64 values of K, within the
// scratch capacity cap (values) at part.
void plan_split(GemmArgs& g, double* part, int64_t cap) {
  g.split = 1;
  g.kc = g.K;
  g.part = nullptr;
  if (!part) return;
  const int64_t tiles = ((g.M + kGemmTile - 1) / kGemmTile) * ((g.N + kGemmTile - 1) / kGemmTile) *
                        g.batch;
  int64_t S = std::min<int64_t>(8, 2048 / std::max<int64_t>(tiles, 1));
  while (S > 1 && (g.K / S < 64 || S * g.batch * g.M * g.N > cap)) --S;
  if (S <= 1) return;
  const int64_t kc = ((g.K + S - 1) / S + 3) & ~(int64_t)3;
  g.split = (g.K + kc - 1) / kc;
  g.kc = kc;
  g.part = part;
  if (g.split <= 1) {
    g.split = 1;
    g.kc = g.K;
    g.part = nullptr;
  }
}

// ------------------------------------------------------------------ device: fit tables
// The tables of one fit of the adaptive loop, from the knots T_a and the
// Gram inverse Z_a of each axis: row i of qt[a] (N_a x n_a) is the
// combination of the p + 1 rows of Z_a picked by the basis functions alive
// at u_i (the pseudo-inverse, transposed), and column i of bt[a] (n_a x N_a)
// holds those basis values, zeros elsewhere (the collocation matrix,
// transposed).  Span rule and basis recurrence as on the host: the largest
// i in [p, n-1] with T[i] <= u, and de Boor's triangular scheme.
struct TabArgs {
  const double* u[3];   // sample parameters in the caller's order
  const double* T[3];   // knots, n + p + 1
  const double* Z[3];   // Gram inverse, n x n
  double* qt[3];
  double* bt[3];
  int32_t N[3], n[3], p[3];
};

__device__ int tab_span(const double* T, int p, int n, double u) {
  int lo = p, hi = n - 1;
  if (T[hi] <= u) return hi;
  while (hi - lo > 1) {                // T[hi] > u; T[lo] <= u unless lo == p
    const int mid = (lo + hi) >> 1;
    if (T[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Z = (L L^T)^-1 of each axis from its banded Cholesky factor (layout as
// on the host, L[j * (p + 1) + d] = L(j, j - d), except that the diagonal
// slot d = 0 holds 1 / L(j, j)): thread c solves L y = e_c (y_j = 0 for
// j < c) and then L^T z = y, into row c of Z (Z is symmetric), keeping the
// last p values of each recurrence in registers.
struct ZinvArgs {
  const double* L[3];
  double* Z[3];
  int32_t n[3], p[3];
  int32_t l_lds;   // the factor is staged in LDS (else read from global memory)
  int32_t y_lds;   // the y rows live in LDS (else in the output row of Z itself)
};

constexpr int kZinvThreads = 16;      // columns per workgroup (their y rows share the LDS)

// L and y in LDS (the recurrences' operands one LDS round trip away), z
// written to global memory once.
template <int P>
__device__ __forceinline__ void zinv_row(const double* L, double* y, double* __restrict__ z, int n,
                                         int c) {
  constexpr int w = P + 1;
  for (int j = 0; j < c; ++j) z[j] = 0.0;
  double win[P + 1];                    // win[d] = y_{j-d} (0 before c)
#pragma unroll
  for (int d = 0; d <= P; ++d) win[d] = 0.0;
#pragma unroll 4
  for (int j = c; j < n; ++j) {
    double v = j == c ? 1.0 : 0.0;
#pragma unroll
    for (int d = P; d >= 1; --d) v -= L[j * w + d] * win[d];
    const double yj = v * L[j * w];
    y[j] = yj;
#pragma unroll
    for (int d = P; d >= 2; --d) win[d] = win[d - 1];
    win[1] = yj;
  }
#pragma unroll
  for (int d = 0; d <= P; ++d) win[d] = 0.0;   // now win[d] = z_{j+d} (0 past n-1)
#pragma unroll 4
  for (int j = n - 1; j >= c; --j) {           // z_j for j < c needs y_j = 0 only
    double v = y[j];
#pragma unroll
    for (int d = 1; d <= P; ++d)
      if (j + d < n) v -= L[(j + d) * w + d] * win[d];
    const double x = v * L[j * w];
    z[j] = x;
#pragma unroll
    for (int d = P; d >= 2; --d) win[d] = win[d - 1];
    win[1] = x;
  }
  for (int j = c - 1; j >= 0; --j) {
    double v = 0.0;
#pragma unroll
    for (int d = 1; d <= P; ++d)
      if (j + d < n) v -= L[(j + d) * w + d] * win[d];
    const double x = v * L[j * w];
    z[j] = x;
#pragma unroll
    for (int d = P; d >= 2; --d) win[d] = win[d - 1];
    win[1] = x;
  }
}

// dynamic LDS: the axis' factor (n (p + 1) values), then one y row of n
// values per thread, as far as the device's LDS holds them.  Without room
// for the y rows, y is kept in the thread's own output row of Z (the
// backward solve reads y_j before it overwrites it with z_j); without room
// for the factor either, the factor is read from global memory.
__global__ __launch_bounds__(kZinvThreads) void zinv_k(ZinvArgs za) {
  extern __shared__ double zsh[];
  const int a = blockIdx.y, c = blockIdx.x * kZinvThreads + threadIdx.x;
  const int n = za.n[a], p = za.p[a];
  if (blockIdx.x * kZinvThreads >= n) return;                  // whole workgroup
  if (za.l_lds) {
    for (int q = threadIdx.x; q < n * (p + 1); q += kZinvThreads) zsh[q] = za.L[a][q];
    __syncthreads();
  }
  if (c >= n) return;
  const double* L = za.l_lds ? zsh : za.L[a];
  double* z = za.Z[a] + (int64_t)c * n;
  double* y = za.y_lds ? zsh + n * (p + 1) + threadIdx.x * n : z;
  switch (p) {
    case 1: zinv_row<1>(L, y, z, n, c); break;
    case 2: zinv_row<2>(L, y, z, n, c); break;
    case 3: zinv_row<3>(L, y, z, n, c); break;
    case 4: zinv_row<4>(L, y, z, n, c); break;
    case 5: zinv_row<5>(L, y, z, n, c); break;
    case 6: zinv_row<6>(L, y, z, n, c); break;
    default: zinv_row<kMaxDegree>(L, y, z, n, c); break;
  }
}

// one wave per sample i of axis blockIdx.y; the lanes run over the n
// control points (rows of Z read along their length, rows of qt written so)
__global__ __launch_bounds__(256) void tables_k(TabArgs ta) {
  const int a = blockIdx.y, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int N = ta.N[a], n = ta.n[a], p = ta.p[a];
  if (i >= N) return;
  const double* T = ta.T[a];
  const double u = ta.u[a][i];
  const int s = tab_span(T, p, n, u);
  double bv[kMaxDegree + 1], left[kMaxDegree + 1], right[kMaxDegree + 1];
  bv[0] = 1.0;
#pragma unroll
  for (int q = 1; q <= kMaxDegree; ++q) {
    if (q > p) break;
    left[q] = u - T[s + 1 - q];
    right[q] = T[s + q] - u;
    double carry = 0.0;
#pragma unroll
    for (int r = 0; r < q; ++r) {
      const double den = right[r + 1] + left[q - r];
      const double t = den != 0.0 ? bv[r] / den : 0.0;
      bv[r] = carry + right[r + 1] * t;
      carry = left[q - r] * t;
    }
    bv[q] = carry;
  }
  const double* Z = ta.Z[a] + (int64_t)(s - p) * n;
  double* qrow = ta.qt[a] + (int64_t)i * n;
  for (int j = lane; j < n; j += 64) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r <= kMaxDegree; ++r)
      if (r <= p) v += bv[r] * Z[(int64_t)r * n + j];
    qrow[j] = v;
    double b = 0.0;
#pragma unroll
    for (int r = 0; r <= kMaxDegree; ++r)
      if (r <= p && j == s - p + r) b = bv[r];
    ta.bt[a][(int64_t)j * N + i] = b;
  }
}

// inv_range = 1 / (max - min) of the samples from the per-block partial
// minima and maxima of minmax_k (1 when the samples are constant): one
// workgroup.
__global__ __launch_bounds__(256) void range_k(const float2* __restrict__ part, int nb,
                                               double* __restrict__ inv_range) {
  __shared__ float lo[256], hi[256];
  float a = __builtin_inff(), b = -__builtin_inff();
  for (int i = threadIdx.x; i < nb; i += 256) {
    a = fminf(a, part[i].x);
    b = fmaxf(b, part[i].y);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o; o >>= 1) {
    if (threadIdx.x < o) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + o]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double range = (double)hi[0] - (double)lo[0];
    *inv_range = range > 0.0 ? 1.0 / range : 1.0;
  }
}

// ------------------------------------------------------------------ host: collocation
// Span rule s = max{ i in [p, n-1] : T[i] <= u }.
int span_of(const double* T, int p, int n, double u) {
  const int s = (int)(std::upper_bound(T + p, T + n, u) - T) - 1;
  return std::min(std::max(s, p), n - 1);
}

// Values of the p+1 basis functions active on span s at u (de Boor's
// triangular scheme: the degree-q values from the degree-(q-1) ones with
// the weights (u - T_i) / (T_{i+q} - T_i), a zero denominator giving 0).
void basis_values(const double* T, int p, int s, double u, double* N) {
  double left[kMaxDegree + 1], right[kMaxDegree + 1];
  N[0] = 1.0;
  for (int q = 1; q <= p; ++q) {
    left[q] = u - T[s + 1 - q];
    right[q] = T[s + q] - u;
    double carry = 0.0;
    for (int r = 0; r < q; ++r) {
      const double den = right[r + 1] + left[q - r];
      const double t = den != 0.0 ? N[r] / den : 0.0;
      N[r] = carry + right[r + 1] * t;
      carry = left[q - r] * t;
    }
    N[q] = carry;
  }
}

// The Cholesky factor of the Gram matrix G = B^T B of the collocation
// matrix B of one axis: G is banded (bandwidth p), G = L L^T with L stored
// by rows, L[j * (p + 1) + d] = L(j, j - d).  The spans and basis values of
// the samples are left in s and Bv ((p + 1) per sample).
mfa_status gram_factor(const double* T, int p, int n, const double* u, int N, int axis,
                       std::vector<double>& L, std::vector<int>& s, std::vector<double>& Bv) {
  const int w = p + 1;
  s.resize(N);
  Bv.resize((size_t)N * w);
  for (int i = 0; i < N; ++i) {
    s[i] = span_of(T, p, n, u[i]);
    basis_values(T, p, s[i], u[i], &Bv[(size_t)i * w]);
  }
  // G[j * w + d] = (B^T B)[j][j - d], d = 0..p
  std::vector<double> G((size_t)n * w, 0.0);
  for (int i = 0; i < N; ++i)
    for (int r1 = 0; r1 <= p; ++r1)
      for (int r2 = 0; r2 <= r1; ++r2)
        G[(size_t)(s[i] - p + r1) * w + (r1 - r2)] += Bv[(size_t)i * w + r1] * Bv[(size_t)i * w + r2];
  double gmax = 0.0;
  for (int j = 0; j < n; ++j) gmax = std::max(gmax, G[(size_t)j * w]);
  // L[j * w + d] = L[j][j - d]
  L.assign((size_t)n * w, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = std::max(0, j - p); k <= j; ++k) {
      double v = G[(size_t)j * w + (j - k)];
      for (int m = std::max(0, j - p); m < k; ++m) v -= L[(size_t)j * w + (j - m)] * L[(size_t)k * w + (k - m)];
      if (k < j) {
        L[(size_t)j * w + (j - k)] = v / L[(size_t)k * w];
      } else {
        if (!(v > 1e-13 * gmax))
          return fail(MFA_E_ARG,
                      "axis %d: the collocation matrix has dependent columns near control point %d "
                      "(a basis function without enough samples: raise res or lower n_ctrl)",
                      axis, j);
        L[(size_t)j * w] = std::sqrt(v);
      }
    }
  return MFA_OK;
}

// Z = (B^T B)^-1 = (L L^T)^-1 (n x n, row-major, symmetric), formed column
// by column (two banded triangular solves per unit vector).
mfa_status gram_inverse(const double* T, int p, int n, const double* u, int N, int axis,
                        std::vector<double>& Z, std::vector<int>& s, std::vector<double>& Bv) {
  const int w = p + 1;
  std::vector<double> L;
  const mfa_status st = gram_factor(T, p, n, u, N, axis, L, s, Bv);
  if (st != MFA_OK) return st;
  Z.resize((size_t)n * n);
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    std::fill(y.begin(), y.end(), 0.0);
    for (int j = c; j < n; ++j) {                        // L y = e_c (y[j] = 0 for j < c)
      double v = j == c ? 1.0 : 0.0;
      for (int m = std::max(c, j - p); m < j; ++m) v -= L[(size_t)j * w + (j - m)] * y[m];
      y[j] = v / L[(size_t)j * w];
    }
    for (int j = n - 1; j >= 0; --j) {                   // L^T x = y (in place)
      double v = y[j];
      for (int m = j + 1; m <= std::min(n - 1, j + p); ++m) v -= L[(size_t)m * w + (m - j)] * y[m];
      y[j] = v / L[(size_t)j * w];
    }
    std::copy(y.begin(), y.end(), Z.begin() + (size_t)c * n);
  }
  return MFA_OK;
}

// Q = (B^T B)^-1 B^T, stored transposed (N x n row-major): row i of Q is the
// combination of the p + 1 rows of Z picked by the non-zeros of row i of B
// (Z is symmetric).
mfa_status pseudo_inverse(const double* T, int p, int n, const double* u, int N, int axis,
                          std::vector<double>& Q) {
  const int w = p + 1;
  std::vector<double> Z, Bv;
  std::vector<int> s;
  const mfa_status st = gram_inverse(T, p, n, u, N, axis, Z, s, Bv);
  if (st != MFA_OK) return st;
  Q.assign((size_t)n * N, 0.0);
  for (int i = 0; i < N; ++i) {
    double* q = &Q[(size_t)i * n];
    for (int r = 0; r <= p; ++r) {
      const double b = Bv[(size_t)i * w + r];
      const double* z = &Z[(size_t)(s[i] - p + r) * n];
      for (int j = 0; j < n; ++j) q[j] += b * z[j];
    }
  }
  return MFA_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The fit's first mode product without the dense pseudo-inverse: per
// fiber (i1, i2) of the samples, Z = B0^T F (p + 1 non-zeros per sample),
// then the two banded triangular solves L y = Z, L^T x = y with the host's
// Cholesky factor of B0^T B0 (bandwidth p), so x = (B0^T B0)^-1 B0^T F, the
// fiber of F x_0 B0+.  The samples are taken in the order of their spans
// (perm), so a control point's sum is complete once a sample past its
// support arrives and it enters the forward solve at once; the backward
// solve runs over the stored y.  One thread per fiber, fibers consecutive
// across the lanes, so every sample and control-point access is one
// coalesced row; the tables (uniform over the lanes) come through the
// scalar cache.  O((p + 1)(N0 + 2 n0)) FP64 operations and 4 N0 + 24 n0
// bytes per fiber, against 2 N0 n0 operations for the dense product.
constexpr int kBand = kMaxDegree + 1;     // window of partial sums (p + 1 <= kBand)
constexpr int kBandUnroll = 8;            // sample loads in flight per thread

__global__ __launch_bounds__(256) void band_fit0_k(const float* __restrict__ f, double* __restrict__ y,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ c0t,
                                                   const double* __restrict__ bv,
                                                   const double* __restrict__ lf,
                                                   const double* __restrict__ inv_d,
                                                   const int32_t* __restrict__ pdeg, int64_t M, int N0,
                                                   int n0) {
  const int64_t fib = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (fib >= M) return;                  // no barriers below
  const int p = pdeg[0], w = p + 1;
  double z[kBand];                       // partial sums of control points cn .. cn + kBand - 1
  double yh[kBand - 1];                  // y[cn - 1 - d] at d
#pragma unroll
  for (int r = 0; r < kBand; ++r) z[r] = 0.0;
#pragma unroll
  for (int d = 0; d < kBand - 1; ++d) yh[d] = 0.0;
  int cn = 0;                            // next control point to solve for
  auto solve_next = [&]() {              // y[cn] = (Z[cn] - sum_d L(cn, cn - d) y[cn - d]) / L(cn, cn)
    double v = z[0];
#pragma unroll
    for (int d = 1; d < kBand; ++d)
      if (d <= p) v -= lf[(int64_t)cn * w + d] * yh[d - 1];   // L(cn, cn - d) = 0 for cn < d
    v *= inv_d[cn];
    y[(int64_t)cn * M + fib] = v;
#pragma unroll
    for (int d = kBand - 2; d > 0; --d) yh[d] = yh[d - 1];
    yh[0] = v;
#pragma unroll
    for (int r = 0; r < kBand - 1; ++r) z[r] = z[r + 1];
    z[kBand - 1] = 0.0;
    ++cn;
  };
  for (int i0 = 0; i0 < N0; i0 += kBandUnroll) {
    float fv[kBandUnroll];             // loads without branches, all in flight together
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) fv[u] = f[(int64_t)perm[min(i0 + u, N0 - 1)] * M + fib];
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) {
      const int i = i0 + u;
      if (i >= N0) break;
      const int c = c0t[i];
      while (cn < c) solve_next();       // no later sample reaches them
      const double v = (double)fv[u];
#pragma unroll
      for (int r = 0; r < kBand; ++r)
        if (r <= p) z[r] = fma(bv[(int64_t)i * w + r], v, z[r]);
    }
  }
  while (cn < n0) solve_next();
  // x[j] = (y[j] - sum_d L(j + d, j) x[j + d]) / L(j, j), from the last
  double xh[kBand - 1];                  // x[j + 1 + d] at d
#pragma unroll
  for (int d = 0; d < kBand - 1; ++d) xh[d] = 0.0;
  for (int j1 = n0 - 1; j1 >= 0; j1 -= kBandUnroll) {
    double yv[kBandUnroll];
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) yv[u] = y[(int64_t)max(j1 - u, 0) * M + fib];
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) {
      const int j = j1 - u;
      if (j < 0) break;
      double v = yv[u];
#pragma unroll
      for (int d = 1; d < kBand; ++d)
        if (d <= p && j + d < n0) v -= lf[(int64_t)(j + d) * w + d] * xh[d - 1];
      v *= inv_d[j];
      y[(int64_t)j * M + fib] = v;
#pragma unroll
      for (int d = kBand - 2; d > 0; --d) xh[d] = xh[d - 1];
      xh[0] = v;
    }
  }
}

// The three mode products of a fit, P = F x_0 B0+ x_1 B1+ x_2 B2+, with the
// tables qt[a] = B_a+ transposed (N_a x n_a).  The first, by far the
// largest (N = N1 N2 columns), runs 32 x 64 tiles per wave (fewer operand
// loads per MFMA); the other two keep 32 x 32 (measured faster there).  Y1 is written transposed,
// [N2][n0 * n1], so that the third product reads its A operand along rows
// of 16 consecutive values.
hipError_t run_fit(const int64_t N[3], const int64_t n[3], const float* values, double* ctrl,
                   const double* const qt[3], double* y0, double* y1, hipStream_t hs,
                   double* split_part = nullptr, int64_t split_cap = 0) {
  GemmArgs g0{n[0], N[1] * N[2], N[0], 1, qt[0], n[0], 0, values, N[1] * N[2], 0, y0,
              N[1] * N[2], 0, 0};
  // Y1 = Y0 x_1 B1+ as its transpose per batch i0, Y1[i2][i0][j1] = sum_i1
  // Y0[i0][i1][i2] B1+[j1][i1]: rows i2 of Y0 as the (transposed) A operand,
  // so that the stores run along j1 (the plain product would store along i2
  // with a stride of n0 n1 values)
  GemmArgs g1{N[2], n[1], N[1], n[0], y0, N[2], N[1] * N[2], qt[1], n[1], 0, y1, n[0] * n[1],
              n[1], 0};
  GemmArgs g2{n[0] * n[1], n[2], N[2], 1, y1, n[0] * n[1], 0, qt[2], n[2], 0, ctrl, n[2], 0, 0};
  plan_split(g1, split_part, split_cap);
  plan_split(g2, split_part, split_cap);
  hipError_t e = gemm<float, true, false, 4>(g0, hs);
  if (e == hipSuccess) e = gemm<double, true>(g1, hs);
  if (e == hipSuccess) e = gemm<double, true>(g2, hs);
  return e;
}

// The spline on the sample grid, Fh = P x_0 B0 x_1 B1 x_2 B2, with the
// collocation tables bt[a] transposed (n_a x N_a); R1 is written transposed
// ([n2][N0 * N1]) for the same reason as Y1 above.  Fh itself is never
// stored: the last product leaves the per-tile row and column maxima of the
// relative error (ErrOut), with rows m = i0 * N1 + i1 and columns i2.
hipError_t run_recon_err(const int64_t N[3], const int64_t n[3], const double* ctrl,
                         const double* const bt[3], double* r0, double* r1, const ErrOut& eo,
                         hipStream_t hs) {
  GemmArgs g0{N[0], n[1] * n[2], n[0], 1, bt[0], N[0], 0, ctrl, n[1] * n[2], 0, r0, n[1] * n[2], 0, 0};
  // transposed per batch i0 like the fit's x_1 product: R1[j2][i0][i1]
  GemmArgs g1{n[2], N[1], n[1], N[0], r0, n[2], n[1] * n[2], bt[1], N[1], 0, r1, N[0] * N[1], N[1], 0};
  GemmArgs g2{N[0] * N[1], N[2], n[2], 1, r1, N[0] * N[1], 0, bt[2], N[2], 0, nullptr, N[2], 0, 0};
  hipError_t e = gemm<double, true>(g0, hs);
  if (e == hipSuccess) e = gemm<double, true>(g1, hs);
  if (e == hipSuccess) e = gemm<double, true, true, kErrNT>(g2, hs, eo);
  return e;
}

// ------------------------------------------------------------------ errors of a fit
constexpr int kRedRows = 64;        // rows per workgroup of max_lead_k
constexpr int kMinMaxBlocks = 2048;

// dst[y * C + c] = max over rows [y * kRedRows, (y + 1) * kRedRows) of
// src[r * C + c] (values >= 0): one thread per column, coalesced.
__global__ __launch_bounds__(256) void max_lead_k(const double* __restrict__ src, int64_t R,
                                                  int64_t C, double* __restrict__ dst) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  const int64_t r0 = (int64_t)blockIdx.y * kRedRows, r1 = min(r0 + (int64_t)kRedRows, R);
  double m = 0.0;
#pragma unroll 16
  for (int64_t r = r0; r < r1; ++r) m = fmax(m, src[r * C + c]);   // loads issued 16 at a time
  dst[blockIdx.y * C + c] = m;
}

// dst[r] = max over c of src[r * C + c]: one wave per row.
__global__ __launch_bounds__(256) void max_row_k(const double* __restrict__ src, int64_t R, int64_t C,
                                                 double* __restrict__ dst) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const int lane = threadIdx.x & 63;
  double m = 0.0;
  for (int64_t c = lane; c < C; c += 64) m = fmax(m, src[row * C + c]);
#pragma unroll
  for (int o = 32; o; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) dst[row] = m;
}

// dst[c] = max over the R rows of src (R x C), by rounds of max_lead_k that
// shrink R by kRedRows through the scratch buffers t0 / t1 (each of
// ceil(R / kRedRows) * C values).
hipError_t max_lead(const double* src, int64_t R, int64_t C, double* t0, double* t1, double* dst,
                    hipStream_t hs) {
  const unsigned gx = (unsigned)((C + 255) / 256);
  for (int round = 0;; ++round) {
    const int64_t Ry = (R + kRedRows - 1) / kRedRows;
    double* out = Ry == 1 ? dst : (round % 2 ? t1 : t0);
    hipLaunchKernelGGL(max_lead_k, dim3(gx, (unsigned)Ry), dim3(256), 0, hs, src, R, C, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || Ry == 1) return e;
    src = out;
    R = Ry;
  }
}

// Per-workgroup (min, max) of the samples, for the data range.
__global__ __launch_bounds__(256) void minmax_k(const float* __restrict__ f, int64_t n,
                                                float2* __restrict__ part) {
  __shared__ float lo[256], hi[256];
  float a = __builtin_inff(), b = -__builtin_inff();
  // up to 3 leading values before a 16-byte boundary, then float4 loads, then the tail
  const int64_t h = min(n, (int64_t)(((16 - ((uintptr_t)f & 15)) & 15) >> 2));
  const int64_t n4 = (n - h) / 4, stride = (int64_t)gridDim.x * 256;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float4* f4 = reinterpret_cast<const float4*>(f + h);
  for (int64_t i = tid; i < n4; i += stride) {
    const float4 v = f4[i];
    a = fminf(a, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
    b = fmaxf(b, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
  }
  if (tid < h) {
    a = fminf(a, f[tid]);
    b = fmaxf(b, f[tid]);
  }
  for (int64_t i = h + 4 * n4 + tid; i < n; i += stride) {
    a = fminf(a, f[i]);
    b = fmaxf(b, f[i]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o; o >>= 1) {
    if (threadIdx.x < o) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + o]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(lo[0], hi[0]);
}

// The x_0 product takes the banded route when the samples have enough
// fibers (res1 res2, one thread each) to hide the latency of its sequential
// solve per fiber and when its bytes take less time than the dense
// product's matrix work, by the rates measured on MI355X: 512^3 -> 192^3
// (2^18 fibers) 0.48 ms banded (3.6 TB/s of its 1.75 GB) against 0.92 ms
// for the GEMM (56 TFLOP/s); at 2^16 fibers (256^3 -> 128^3) the banded
// route was slower, 0.26 against 0.17 ms.
constexpr int64_t kBandMinFibers = int64_t(1) << 17;
constexpr double kBandBytesPerS = 3.6e12, kGemmFlopPerS = 55e12;

bool band_route(const int32_t res[3], const int32_t n_ctrl[3]) {
  const double M = (double)res[1] * res[2], N0 = res[0], n0 = n_ctrl[0];
  if (M < (double)kBandMinFibers) return false;
  const double t_band = (4.0 * N0 + 24.0 * n0) * M / kBandBytesPerS;   // F; y out, in; x out
  const double t_gemm = 2.0 * n0 * N0 * M / kGemmFlopPerS;
  return t_band < t_gemm;
}

// Workspace layout: with the banded route, the tables of axis 0 (sample
// order, control point of each support, basis values, Cholesky factor rows,
// reciprocal diagonal, degree), else Q0; Q1, Q2 (B_a+ transposed, FP64);
// then Y0 = F x_0 B0+ (n0 x N1 x N2) and Y1 = Y0 x_1 B1+ (stored N2 x n0 x n1).
struct EncodeLayout {
  size_t perm, c0, bv, lf, inv_d, pdeg, q[3], y0, y1, total;
  bool band;
};

EncodeLayout encode_layout(const int32_t res[3], const int32_t n_ctrl[3]) {
  EncodeLayout L{};
  size_t o = 0;
  const size_t N0 = res[0], n0 = n_ctrl[0], w = kMaxDegree + 1;
  L.band = band_route(res, n_ctrl);
  if (L.band) {
    L.perm = o;
    o += align256(4 * N0);
    L.c0 = o;
    o += align256(4 * N0);
    L.bv = o;
    o += align256(8 * N0 * w);
    L.lf = o;
    o += align256(8 * n0 * w);
    L.inv_d = o;
    o += align256(8 * n0);
    L.pdeg = o;
    o += 256;
  }
  for (int a = L.band ? 1 : 0; a < 3; ++a) {
    L.q[a] = o;
    o += align256(8 * (size_t)n_ctrl[a] * (size_t)res[a]);
  }
  L.y0 = o;
  o += align256(8 * (size_t)n_ctrl[0] * (size_t)res[1] * (size_t)res[2]);
  L.y1 = o;
  o += align256(8 * (size_t)n_ctrl[0] * (size_t)n_ctrl[1] * (size_t)res[2]);
  L.total = o;
  return L;
}

constexpr int32_t kMaxEncodeRes = 1 << 16;

mfa_status check_sizes(const int32_t res[3], const int32_t n_ctrl[3], const int32_t* degree) {
  if (!res || !n_ctrl) return fail(MFA_E_ARG, "null res / n_ctrl");
  for (int a = 0; a < 3; ++a) {
    const int p = degree ? degree[a] : 1;
    if (degree && (p < 1 || p > kMaxDegree))
      return fail(MFA_E_ARG, "axis %d: degree %d outside [1, %d]", a, p, kMaxDegree);
    if (n_ctrl[a] < p + 1 || n_ctrl[a] > kMaxEncodeRes)
      return fail(MFA_E_ARG, "axis %d: n_ctrl %d outside [degree + 1, %d]", a, n_ctrl[a], kMaxEncodeRes);
    if (res[a] < n_ctrl[a] || res[a] > kMaxEncodeRes)
      return fail(MFA_E_ARG, "axis %d: res %d outside [n_ctrl, %d]", a, res[a], kMaxEncodeRes);
  }
  return MFA_OK;
}

}  // namespace
}  // namespace mfa

using namespace mfa;

extern "C" mfa_status mfa_encode_workspace(const int32_t res[3], const int32_t n_ctrl[3],
                                           int64_t* bytes) {
  if (!bytes) return fail(MFA_E_ARG, "null bytes");
  mfa_status st = check_sizes(res, n_ctrl, nullptr);
  if (st != MFA_OK) return st;
  *bytes = (int64_t)encode_layout(res, n_ctrl).total;
  return MFA_OK;
}

extern "C" mfa_status mfa_encode_plan(const int32_t res[3], const double* const axis_u[3],
                                      const int32_t degree[3], const int32_t n_ctrl[3],
                                      const double* const knots[3], void* work, int64_t work_bytes,
                                      void* stream) {
  if (!degree) return fail(MFA_E_ARG, "null degree");
  mfa_status st = check_sizes(res, n_ctrl, degree);
  if (st != MFA_OK) return st;
  if (!axis_u || !work) return fail(MFA_E_ARG, "null axis_u / work");
  const EncodeLayout lay = encode_layout(res, n_ctrl);
  if (work_bytes < (int64_t)lay.total)
    return fail(MFA_E_ARG, "workspace of %lld bytes, %lld needed", (long long)work_bytes,
                (long long)lay.total);
  std::vector<double> Q[3];
  // axis 0: the samples in span order, their supports and basis values, the
  // Cholesky factor of the Gram matrix and its reciprocal diagonal
  std::vector<int32_t> perm, c0s;
  std::vector<double> bvs, lf, inv_d;
  int32_t p0 = degree[0];
  for (int a = 0; a < 3; ++a) {
    const int p = degree[a], n = n_ctrl[a], N = res[a];
    if (!axis_u[a]) return fail(MFA_E_ARG, "axis %d: null parameter table", a);
    for (int i = 0; i < N; ++i)
      if (!(axis_u[a][i] >= 0.0 && axis_u[a][i] <= 1.0))
        return fail(MFA_E_ARG, "axis %d: parameter %d = %g outside [0, 1]", a, i, axis_u[a][i]);
    std::vector<double> T(n + p + 1);
    if (knots && knots[a]) {
      st = check_knots(knots[a], n, p, 0, a);
      if (st != MFA_OK) return st;
      std::copy(knots[a], knots[a] + n + p + 1, T.begin());
    } else {
      default_knots(n, p, T.data());
    }
    if (a == 0 && lay.band) {
      std::vector<int> s;
      std::vector<double> Bv;
      st = gram_factor(T.data(), p, n, axis_u[a], N, a, lf, s, Bv);
      if (st != MFA_OK) return st;
      const int w = p + 1;
      perm.resize(N);
      for (int i = 0; i < N; ++i) perm[i] = i;
      std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return s[x] < s[y]; });
      c0s.resize(N);
      bvs.resize((size_t)N * w);
      for (int k = 0; k < N; ++k) {
        c0s[k] = s[perm[k]] - p;
        std::copy(&Bv[(size_t)perm[k] * w], &Bv[(size_t)perm[k] * w] + w, &bvs[(size_t)k * w]);
      }
      inv_d.resize(n);
      for (int j = 0; j < n; ++j) inv_d[j] = 1.0 / lf[(size_t)j * w];
      continue;
    }
    st = pseudo_inverse(T.data(), p, n, axis_u[a], N, a, Q[a]);
    if (st != MFA_OK) return st;
  }
  hipStream_t hs = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(work);
  struct Up {
    size_t off;
    const void* src;
    size_t bytes;
  };
  std::vector<Up> ups;
  if (lay.band)
    ups = {{lay.perm, perm.data(), perm.size() * 4},    {lay.c0, c0s.data(), c0s.size() * 4},
           {lay.bv, bvs.data(), bvs.size() * 8},        {lay.lf, lf.data(), lf.size() * 8},
           {lay.inv_d, inv_d.data(), inv_d.size() * 8}, {lay.pdeg, &p0, 4}};
  else
    ups = {{lay.q[0], Q[0].data(), Q[0].size() * 8}};
  ups.push_back({lay.q[1], Q[1].data(), Q[1].size() * 8});
  ups.push_back({lay.q[2], Q[2].data(), Q[2].size() * 8});
  for (const Up& u : ups) {
    hipError_t e = hipMemcpyAsync(wb + u.off, u.src, u.bytes, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "encode: table upload");
  }
  // the host tables must outlive their upload: wait for it (and for the
  // work queued before it on the stream)
  hipError_t e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return hip_fail(e, "encode: pseudo-inverse upload");
  return MFA_OK;
}

extern "C" mfa_status mfa_encode_apply(const int32_t res[3], const int32_t n_ctrl[3],
                                       const float* values, double* ctrl, void* work,
                                       int64_t work_bytes, void* stream) {
  mfa_status st = check_sizes(res, n_ctrl, nullptr);
  if (st != MFA_OK) return st;
  if (!values || !ctrl || !work) return fail(MFA_E_ARG, "null values / ctrl / work");
  const EncodeLayout lay = encode_layout(res, n_ctrl);
  if (work_bytes < (int64_t)lay.total)
    return fail(MFA_E_ARG, "workspace of %lld bytes, %lld needed", (long long)work_bytes,
                (long long)lay.total);
  hipStream_t hs = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(work);
  auto at = [&](size_t off) { return reinterpret_cast<double*>(wb + off); };
  double* y0 = at(lay.y0);
  double* y1 = at(lay.y1);
  const int64_t N0 = res[0], N1 = res[1], N2 = res[2];
  const int64_t n0 = n_ctrl[0], n1 = n_ctrl[1], n2 = n_ctrl[2];
  if (!lay.band) {                       // three GEMMs with the tables B_a+ transposed (N_a x n_a)
    const double* dq[3] = {at(lay.q[0]), at(lay.q[1]), at(lay.q[2])};
    const int64_t N[3] = {N0, N1, N2}, n[3] = {n0, n1, n2};
    hipError_t e = run_fit(N, n, values, ctrl, dq, y0, y1, hs);
    if (e != hipSuccess) return hip_fail(e, "encode: GEMM launch");
    return MFA_OK;
  }
  // Y0 = F x_0 B0+ by the banded route, then the x_1 and x_2 products as
  // GEMMs with the tables B_a+ transposed (N_a x n_a)
  const int64_t M = N1 * N2;
  hipLaunchKernelGGL(band_fit0_k, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, hs, values, y0,
                     reinterpret_cast<const int32_t*>(wb + lay.perm),
                     reinterpret_cast<const int32_t*>(wb + lay.c0), at(lay.bv), at(lay.lf),
                     at(lay.inv_d), reinterpret_cast<const int32_t*>(wb + lay.pdeg), M, (int)N0,
                     (int)n0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "encode: banded fit launch");
  GemmArgs g1{N2, n1, N1, n0, y0, N2, N1 * N2, at(lay.q[1]), n1, 0, y1, n0 * n1, n1, 0};
  GemmArgs g2{n0 * n1, n2, N2, 1, y1, n0 * n1, 0, at(lay.q[2]), n2, 0, ctrl, n2, 0, 0};
  plan_split(g1, nullptr, 0);
  plan_split(g2, nullptr, 0);
  e = gemm<double, true>(g1, hs);
  if (e == hipSuccess) e = gemm<double, true>(g2, hs);
  if (e != hipSuccess) return hip_fail(e, "encode: GEMM launch");
  return MFA_OK;
}

extern "C" mfa_status mfa_encode_grid(const int32_t res[3], const double* const axis_u[3],
                                      const float* values, const int32_t degree[3],
                                      const int32_t n_ctrl[3], const double* const knots[3],
                                      double* ctrl, void* work, int64_t work_bytes, void* stream) {
  if (!values || !ctrl) return fail(MFA_E_ARG, "null values / ctrl");
  mfa_status st = mfa_encode_plan(res, axis_u, degree, n_ctrl, knots, work, work_bytes, stream);
  if (st != MFA_OK) return st;
  return mfa_encode_apply(res, n_ctrl, values, ctrl, work, work_bytes, stream);
}

namespace mfa {
namespace {

// Workspace of the adaptive loop, sized for max_ctrl control points per
// axis: the tables, the intermediates of a fit and of a reconstruction, the
// per-tile error maxima (rows m = i0 * N1 + i1 of the last reconstruction
// product, columns i2), their reduction scratch, the three marginals and the
// split-K partial products of the fit (a split product has at most 2048
// tiles of 32 x 32 over all its chunks, so 2^21 values always suffice), the
// sample parameters, the staging area of each fit's knots and Gram factors
// (packed, at most max_ctrl + kMaxDegree + 1 and (kMaxDegree + 1) max_ctrl
// values per axis), the Gram inverses (packed, at most max_ctrl^2 per axis)
// and 1 / data range.
struct AdaptLayout {
  size_t qt[3], bt[3], y0, y1, r0, r1, rowpart, colpart, rowmax, red0, red1, marg, mm, part, u, stage,
      z, inv, total;
  int64_t part_cap;
};

constexpr int64_t kSplitCap = int64_t(1) << 21;

AdaptLayout adapt_layout(const int32_t res[3], const int32_t nm[3]) {
  AdaptLayout L{};
  const size_t N0 = res[0], N1 = res[1], N2 = res[2], m0 = nm[0], m1 = nm[1], m2 = nm[2];
  const size_t M = N0 * N1, tm = (M + kGemmTile - 1) / kGemmTile, tn = (N2 + 16 * kErrNT - 1) / (16 * kErrNT);
  auto up = [](size_t v) { return (v + kRedRows - 1) / kRedRows; };
  const size_t red = std::max({up(tm) * N2, tn > (size_t)kRedRows ? up(tn) * M : 0, up(N0) * N1});
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  for (int a = 0; a < 3; ++a) L.qt[a] = take(8 * (size_t)res[a] * (size_t)nm[a]);
  for (int a = 0; a < 3; ++a) L.bt[a] = take(8 * (size_t)res[a] * (size_t)nm[a]);
  L.y0 = take(8 * m0 * N1 * N2);
  L.y1 = take(8 * N2 * m0 * m1);
  L.r0 = take(8 * N0 * m1 * m2);
  L.r1 = take(8 * m2 * M);
  L.rowpart = take(8 * tn * M);
  L.colpart = take(8 * tm * N2);
  L.rowmax = take(8 * M);
  L.red0 = take(8 * red);
  L.red1 = take(8 * red);
  L.marg = take(8 * (N0 + N1 + N2));
  L.mm = take(sizeof(float2) * kMinMaxBlocks);
  L.part_cap = std::min<int64_t>(kSplitCap, 8 * (int64_t)(m0 * m1 * N2));
  L.part = take(8 * (size_t)L.part_cap);
  L.u = take(8 * (N0 + N1 + N2));
  L.stage = take(8 * (m0 + m1 + m2 + 3 * (kMaxDegree + 1) + (kMaxDegree + 1) * (m0 + m1 + m2)));
  L.z = take(8 * (m0 * m0 + m1 * m1 + m2 * m2));
  L.inv = take(8);
  L.total = o;
  return L;
}

// Dynamic LDS a workgroup may take on the current device (read once per
// device).
hipError_t device_lds_limit(size_t* bytes) {
  static std::atomic<int> limit[64];     // zero: not read yet
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int v = limit[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (v <= 0) return hipErrorInvalidValue;
    limit[dev].store(v, std::memory_order_relaxed);
  }
  *bytes = (size_t)v;
  return hipSuccess;
}

mfa_status check_adaptive(const int32_t res[3], const int32_t degree[3], const int32_t n_init[3],
                          const int32_t max_ctrl[3]) {
  if (!res || !degree || !n_init || !max_ctrl) return fail(MFA_E_ARG, "null res / degree / n_init / max_ctrl");
  for (int a = 0; a < 3; ++a) {
    if (degree[a] < 1 || degree[a] > kMaxDegree)
      return fail(MFA_E_ARG, "axis %d: degree %d outside [1, %d]", a, degree[a], kMaxDegree);
    if (n_init[a] < degree[a] + 1 || max_ctrl[a] < n_init[a] || max_ctrl[a] > res[a] ||
        res[a] > kMaxEncodeRes)
      return fail(MFA_E_ARG, "axis %d: need degree + 1 <= n_init <= max_ctrl <= res <= %d", a,
                  kMaxEncodeRes);
  }
  return MFA_OK;
}

}  // namespace
}  // namespace mfa

extern "C" mfa_status mfa_encode_adaptive_workspace(const int32_t res[3], const int32_t max_ctrl[3],
                                                    int64_t* bytes) {
  if (!bytes || !res || !max_ctrl) return fail(MFA_E_ARG, "null argument");
  const int32_t one[3] = {1, 1, 1}, n1[3] = {2, 2, 2};
  mfa_status st = check_adaptive(res, one, n1, max_ctrl);
  if (st != MFA_OK) return st;
  *bytes = (int64_t)adapt_layout(res, max_ctrl).total;
  return MFA_OK;
}

extern "C" mfa_status mfa_encode_adaptive(const int32_t res[3], const double* const axis_u[3],
                                          const float* values, const int32_t degree[3],
                                          const int32_t n_init[3], const int32_t max_ctrl[3],
                                          double e_max, int32_t max_fits, double* const knots_out[3],
                                          int32_t n_out[3], double* ctrl, int64_t ctrl_capacity,
                                          double* history, int32_t* n_fits, void* work,
                                          int64_t work_bytes, void* stream) {
  mfa_status st = check_adaptive(res, degree, n_init, max_ctrl);
  if (st != MFA_OK) return st;
  if (!axis_u || !values || !knots_out || !n_out || !ctrl || !work || !n_fits)
    return fail(MFA_E_ARG, "null axis_u / values / knots_out / n_out / ctrl / work / n_fits");
  if (!(e_max > 0.0) || !std::isfinite(e_max)) return fail(MFA_E_ARG, "e_max must be finite and > 0");
  if (max_fits < 1) return fail(MFA_E_ARG, "max_fits must be >= 1");
  if (ctrl_capacity < (int64_t)max_ctrl[0] * max_ctrl[1] * max_ctrl[2])
    return fail(MFA_E_ARG, "ctrl capacity %lld < max_ctrl product", (long long)ctrl_capacity);
  const AdaptLayout lay = adapt_layout(res, max_ctrl);
  if (work_bytes < (int64_t)lay.total)
    return fail(MFA_E_ARG, "workspace of %lld bytes, %lld needed", (long long)work_bytes,
                (long long)lay.total);
  std::vector<double> us[3];
  for (int a = 0; a < 3; ++a) {
    if (!axis_u[a] || !knots_out[a]) return fail(MFA_E_ARG, "axis %d: null table", a);
    for (int i = 0; i < res[a]; ++i)
      if (!(axis_u[a][i] >= 0.0 && axis_u[a][i] <= 1.0))
        return fail(MFA_E_ARG, "axis %d: parameter %d = %g outside [0, 1]", a, i, axis_u[a][i]);
    us[a].assign(axis_u[a], axis_u[a] + res[a]);
    std::sort(us[a].begin(), us[a].end());
  }
  hipStream_t hs = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(work);
  auto at = [&](size_t off) { return reinterpret_cast<double*>(wb + off); };
  // an error return after an upload from host vectors of this call waits
  // for the stream first, so no copy still reads from a destroyed vector
  auto bail = [&](mfa_status st) {
    (void)hipStreamSynchronize(hs);
    return st;
  };
  const int64_t N[3] = {res[0], res[1], res[2]};
  const int64_t rows = N[0] * N[1];
  const int64_t tm = (rows + kGemmTile - 1) / kGemmTile, tn = (N[2] + 16 * kErrNT - 1) / (16 * kErrNT);
  if ((tm + kRedRows - 1) / kRedRows > 65535)
    return fail(MFA_E_ARG, "res0 * res1 above %lld", 65535LL * kRedRows * kGemmTile);
  // sample parameters on the device, in the caller's order
  std::vector<double> hu(N[0] + N[1] + N[2]);
  const double* du[3] = {at(lay.u), at(lay.u) + N[0], at(lay.u) + N[0] + N[1]};
  for (int a = 0; a < 3; ++a) std::copy(axis_u[a], axis_u[a] + res[a], hu.begin() + (du[a] - du[0]));
  hipError_t e = hipMemcpyAsync(at(lay.u), hu.data(), hu.size() * 8, hipMemcpyHostToDevice, hs);
  if (e != hipSuccess) return hip_fail(e, "encode: parameter upload");
  // data range, reduced on the device (the error products read 1 / range there)
  float2* mm = reinterpret_cast<float2*>(wb + lay.mm);
  hipLaunchKernelGGL(minmax_k, dim3(kMinMaxBlocks), dim3(256), 0, hs, values, rows * N[2], mm);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(range_k, dim3(1), dim3(256), 0, hs, mm, kMinMaxBlocks, at(lay.inv));
    e = hipGetLastError();
  }
  if (e != hipSuccess) return bail(hip_fail(e, "encode: data range"));
  // initial knots: clamped uniform with n_init control points
  std::vector<double> T[3];
  for (int a = 0; a < 3; ++a) {
    T[a].resize(n_init[a] + degree[a] + 1);
    default_knots(n_init[a], degree[a], T[a].data());
  }
  std::vector<double> Lg[3], Bv[3], stage, marg(N[0] + N[1] + N[2]);
  std::vector<int> spans[3];
  double* dmarg = at(lay.marg);
  const ErrOut eo{values, N[2], at(lay.inv), at(lay.rowpart), at(lay.colpart)};
  int fits = 0;
  for (;;) {
    int64_t n[3];
    for (int a = 0; a < 3; ++a) n[a] = (int64_t)T[a].size() - degree[a] - 1;
    // the Gram factors on the host (banded, O(res p^2) per axis); the device
    // inverts them and forms the tables
    for (int a = 0; a < 3; ++a) {
      const mfa_status sa = gram_factor(T[a].data(), degree[a], (int)n[a], axis_u[a], res[a], a, Lg[a],
                                        spans[a], Bv[a]);
      if (sa != MFA_OK) return bail(sa);    // the parameter upload has its source in hu
    }
    // knots and Gram factors in one copy (the previous pass ended with a
    // synchronisation, so stage is free to reuse)
    TabArgs ta{};
    ZinvArgs za{};
    stage.clear();
    for (int a = 0; a < 3; ++a) {
      ta.T[a] = at(lay.stage) + stage.size();
      stage.insert(stage.end(), T[a].begin(), T[a].end());
    }
    for (int a = 0; a < 3; ++a) {
      za.L[a] = at(lay.stage) + stage.size();
      const size_t o = stage.size();
      stage.insert(stage.end(), Lg[a].begin(), Lg[a].end());
      for (int64_t j = 0; j < n[a]; ++j) stage[o + j * (degree[a] + 1)] = 1.0 / stage[o + j * (degree[a] + 1)];
    }
    e = hipMemcpyAsync(at(lay.stage), stage.data(), stage.size() * 8, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return bail(hip_fail(e, "encode: table upload"));
    int maxN = 0, maxn = 0;
    int64_t zo = 0;
    for (int a = 0; a < 3; ++a) {
      za.Z[a] = at(lay.z) + zo;
      za.n[a] = (int32_t)n[a];
      za.p[a] = degree[a];
      zo += n[a] * n[a];
      maxn = std::max(maxn, (int)n[a]);
      ta.Z[a] = za.Z[a];
      ta.u[a] = du[a];
      ta.qt[a] = at(lay.qt[a]);
      ta.bt[a] = at(lay.bt[a]);
      ta.N[a] = res[a];
      ta.n[a] = (int32_t)n[a];
      ta.p[a] = degree[a];
      maxN = std::max(maxN, res[a]);
    }
    // LDS of the inversion: factor and y rows, else the factor alone, else none
    size_t lds_l = 0, lds_y = 0;
    for (int a = 0; a < 3; ++a) {
      lds_l = std::max(lds_l, (size_t)n[a] * (degree[a] + 1) * 8);
      lds_y = std::max(lds_y, (size_t)n[a] * (degree[a] + 1 + kZinvThreads) * 8);
    }
    size_t lds_limit = 0;
    e = device_lds_limit(&lds_limit);
    if (e != hipSuccess) return bail(hip_fail(e, "encode: device LDS size"));
    za.y_lds = lds_y <= lds_limit;
    za.l_lds = lds_l <= lds_limit;
    const size_t lds = za.y_lds ? lds_y : (za.l_lds ? lds_l : 0);
    hipLaunchKernelGGL(zinv_k, dim3((unsigned)((maxn + kZinvThreads - 1) / kZinvThreads), 3),
                       dim3(kZinvThreads), lds, hs, za);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(tables_k, dim3((unsigned)((maxN + 3) / 4), 3), dim3(256), 0, hs, ta);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return bail(hip_fail(e, "encode: tables"));
    const double* qt[3] = {at(lay.qt[0]), at(lay.qt[1]), at(lay.qt[2])};
    const double* bt[3] = {at(lay.bt[0]), at(lay.bt[1]), at(lay.bt[2])};
    e = run_fit(N, n, values, ctrl, qt, at(lay.y0), at(lay.y1), hs, at(lay.part), lay.part_cap);
    if (e == hipSuccess) e = run_recon_err(N, n, ctrl, bt, at(lay.r0), at(lay.r1), eo, hs);
    // marginals: m0[i0], m1[i1] from the row maxima over i2, m2[i2] over all rows
    if (e == hipSuccess) e = max_lead(eo.rowpart, tn, rows, at(lay.red0), at(lay.red1), at(lay.rowmax), hs);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(max_row_k, dim3((unsigned)((N[0] + 3) / 4)), dim3(256), 0, hs, at(lay.rowmax),
                         N[0], N[1], dmarg);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = max_lead(at(lay.rowmax), N[0], N[1], at(lay.red0), at(lay.red1), dmarg + N[0], hs);
    if (e == hipSuccess)
      e = max_lead(eo.colpart, tm, N[2], at(lay.red0), at(lay.red1), dmarg + N[0] + N[1], hs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(marg.data(), dmarg, marg.size() * 8, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return bail(hip_fail(e, "encode: adaptive fit"));
    // largest error per sample index of each axis
    const double* m[3] = {marg.data(), marg.data() + N[0], marg.data() + N[0] + N[1]};
    double emax = 0.0;
    for (int64_t i = 0; i < N[0]; ++i) emax = std::max(emax, m[0][i]);
    if (history) {
      history[4 * fits + 0] = (double)n[0];
      history[4 * fits + 1] = (double)n[1];
      history[4 * fits + 2] = (double)n[2];
      history[4 * fits + 3] = emax;
    }
    ++fits;
    // spans to halve: largest error over their samples above e_max, and a
    // sample parameter in each half; at most max_ctrl - n per axis (the
    // largest errors first, then the lower span)
    std::vector<double> mids[3];
    bool grow = false;
    for (int a = 0; a < 3; ++a) {
      const int p = degree[a], nsp = (int)n[a] - p;
      std::vector<double> es(nsp, 0.0);
      for (int i = 0; i < res[a]; ++i) {
        const int j = span_of(T[a].data(), p, (int)n[a], axis_u[a][i]) - p;
        es[j] = std::max(es[j], m[a][i]);
      }
      std::vector<std::pair<double, int>> cand;
      for (int j = 0; j < nsp; ++j) {
        const double t0 = T[a][p + j], t1 = T[a][p + j + 1], mid = 0.5 * (t0 + t1);
        if (!(es[j] > e_max)) continue;
        const auto lo_it = std::lower_bound(us[a].begin(), us[a].end(), t0);
        const bool left = lo_it != us[a].end() && *lo_it < mid;
        const auto mid_it = std::lower_bound(us[a].begin(), us[a].end(), mid);
        const bool right = mid_it != us[a].end() && *mid_it <= t1;
        if (left && right) cand.push_back({es[j], j});
      }
      const size_t room = (size_t)(max_ctrl[a] - n[a]);
      if (cand.size() > room) {
        std::stable_sort(cand.begin(), cand.end(),
                         [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                           return x.first > y.first;
                         });
        cand.resize(room);
      }
      for (const auto& c : cand) mids[a].push_back(0.5 * (T[a][p + c.second] + T[a][p + c.second + 1]));
      grow |= !mids[a].empty();
    }
    if (!grow || fits >= max_fits) break;
    for (int a = 0; a < 3; ++a) {
      T[a].insert(T[a].end(), mids[a].begin(), mids[a].end());
      std::sort(T[a].begin(), T[a].end());
    }
  }
  for (int a = 0; a < 3; ++a) {
    n_out[a] = (int32_t)T[a].size() - degree[a] - 1;
    std::copy(T[a].begin(), T[a].end(), knots_out[a]);
  }
  *n_fits = fits;
  return MFA_OK;
}
