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

#include <algorithm>
#include <cmath>
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
};

constexpr int kGemmBlock = 256;   // 4 waves, each computing its own C tile
constexpr int kGemmTile = 32;     // C tile per wave: 2 x 2 MFMA blocks of 16 x 16

// One wave per 32 x 32 tile of C; tiles are numbered with the M tile
// fastest, so the waves of a workgroup share the columns of B they read.
// Per step of 4 along K each lane supplies A(m0 + 16t + lane % 16, k) and
// B(k, n0 + 16u + lane % 16) with k = k0 + lane / 16, and the MFMA leaves
// element (i, j) of a 16 x 16 block in lane j + 16 * (i % 4), register
// i / 4.  Lanes past the last row of A or column of B read the last one
// instead (in bounds): they only feed outputs that are not stored, so the
// main loop has no predicates; the K tail runs one step with zeros past K.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;   // global-memory pointer

constexpr int kGemmUnroll = 4;    // K steps whose loads are issued together

template <typename TB, bool TRANS_A>
__global__ __launch_bounds__(kGemmBlock) void gemm_f64_k(const double* __restrict__ gA,
                                                         const TB* __restrict__ gB,
                                                         double* __restrict__ gC, GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (kGemmBlock / 64) + (threadIdx.x >> 6);
  const int64_t tm = (g.M + kGemmTile - 1) / kGemmTile, tn = (g.N + kGemmTile - 1) / kGemmTile;
  if (w >= tm * tn * g.batch) return;                  // whole wave
  const int64_t im = w % tm, rest = w / tm, jn = rest % tn, b = rest / tn;
  const int c16 = lane & 15, q = lane >> 4;
  const int64_t m0 = im * kGemmTile, n0 = jn * kGemmTile;
  const double* A0 = gA + b * g.sA;
  const TB* B0 = gB + b * g.sB;
  gptr<double> pa[2];
  gptr<TB> pb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t m = min(m0 + 16 * t + c16, g.M - 1), n = min(n0 + 16 * t + c16, g.N - 1);
    pa[t] = (gptr<double>)(TRANS_A ? A0 + (int64_t)q * g.lda + m : A0 + m * g.lda + q);
    pb[t] = (gptr<TB>)(B0 + (int64_t)q * g.ldb + n);
  }
  const int64_t step_a = TRANS_A ? 4 * g.lda : 4, step_b = 4 * g.ldb;
  v4d acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = v4d{0.0, 0.0, 0.0, 0.0};
  auto mma = [&](const double (&a)[2], const double (&bv)[2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bv[u], acc[t][u], 0, 0, 0);
  };
  const int64_t kfull = g.K & ~(int64_t)3;
  int64_t k0 = 0;
  for (; k0 + 4 * kGemmUnroll <= kfull; k0 += 4 * kGemmUnroll) {
    double a[kGemmUnroll][2];
    TB bt[kGemmUnroll][2];
#pragma unroll
    for (int s = 0; s < kGemmUnroll; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[s][t] = pa[t][s * step_a];
        bt[s][t] = pb[t][s * step_b];
      }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      pa[t] += kGemmUnroll * step_a;
      pb[t] += kGemmUnroll * step_b;
    }
#pragma unroll
    for (int s = 0; s < kGemmUnroll; ++s) {
      const double bv[2] = {(double)bt[s][0], (double)bt[s][1]};
      mma(a[s], bv);
    }
  }
  for (; k0 < kfull; k0 += 4) {
    double a[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = *pa[t];
      bv[t] = (double)*pb[t];
      pa[t] += step_a;
      pb[t] += step_b;
    }
    mma(a, bv);
  }
  if (kfull < g.K) {
    const bool kin = kfull + q < g.K;
    double a[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = kin ? *pa[t] : 0.0;
      bv[t] = kin ? (double)*pb[t] : 0.0;
    }
    mma(a, bv);
  }
  double* __restrict__ C = gC + b * g.sC;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + 16 * t + q + 4 * r, n = n0 + 16 * u + c16;
        if (m < g.M && n < g.N) C[g.c_trans ? n * g.ldc + m : m * g.ldc + n] = acc[t][u][r];
      }
}

template <typename TB, bool TRANS_A>
hipError_t gemm(const GemmArgs& g, hipStream_t st) {
  const int64_t tiles = ((g.M + kGemmTile - 1) / kGemmTile) * ((g.N + kGemmTile - 1) / kGemmTile) *
                        g.batch;
  const int64_t blocks = (tiles + kGemmBlock / 64 - 1) / (kGemmBlock / 64);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_f64_k<TB, TRANS_A>), dim3((unsigned)blocks), dim3(kGemmBlock), 0, st, g.A,
                     static_cast<const TB*>(g.B), g.C, g);
  return hipGetLastError();
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

// Q = (B^T B)^-1 B^T, stored transposed (N x n row-major), for the collocation matrix B of one
// axis: the Gram matrix is banded (bandwidth p), factorised as L L^T, and
// each column B^T e_i (non-zero on rows s_i - p .. s_i) is solved for.
mfa_status pseudo_inverse(const double* T, int p, int n, const double* u, int N, int axis,
                          std::vector<double>& Q, std::vector<double>* Bt = nullptr) {
  const int w = p + 1;
  std::vector<int> s(N);
  std::vector<double> Bv((size_t)N * w);
  for (int i = 0; i < N; ++i) {
    s[i] = span_of(T, p, n, u[i]);
    basis_values(T, p, s[i], u[i], &Bv[(size_t)i * w]);
  }
  if (Bt) {                                   // collocation matrix, transposed: Bt[j * N + i]
    Bt->assign((size_t)n * N, 0.0);
    for (int i = 0; i < N; ++i)
      for (int r = 0; r <= p; ++r) (*Bt)[(size_t)(s[i] - p + r) * N + i] = Bv[(size_t)i * w + r];
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
  std::vector<double> L((size_t)n * w, 0.0);
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
  Q.assign((size_t)n * N, 0.0);
  std::vector<double> y(n);
  for (int i = 0; i < N; ++i) {
    const int j0 = s[i] - p;
    std::fill(y.begin(), y.end(), 0.0);
    for (int j = j0; j < n; ++j) {                       // L y = B^T e_i
      double v = (j <= s[i]) ? Bv[(size_t)i * w + (j - j0)] : 0.0;
      for (int m = std::max(j0, j - p); m < j; ++m) v -= L[(size_t)j * w + (j - m)] * y[m];
      y[j] = v / L[(size_t)j * w];
    }
    for (int j = n - 1; j >= 0; --j) {                   // L^T x = y (in place)
      double v = y[j];
      for (int m = j + 1; m <= std::min(n - 1, j + p); ++m) v -= L[(size_t)m * w + (m - j)] * y[m];
      y[j] = v / L[(size_t)j * w];
    }
    for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = y[j];
  }
  return MFA_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The three mode products of a fit, P = F x_0 B0+ x_1 B1+ x_2 B2+, with the
// tables qt[a] = B_a+ transposed (N_a x n_a).  Y1 is written transposed,
// [N2][n0 * n1], so that the third product reads its A operand along rows
// of 16 consecutive values.
hipError_t run_fit(const int64_t N[3], const int64_t n[3], const float* values, double* ctrl,
                   const double* const qt[3], double* y0, double* y1, hipStream_t hs) {
  GemmArgs g0{n[0], N[1] * N[2], N[0], 1, qt[0], n[0], 0, values, N[1] * N[2], 0, y0,
              N[1] * N[2], 0, 0};
  GemmArgs g1{n[1], N[2], N[1], n[0], qt[1], n[1], 0, y0, N[2], N[1] * N[2], y1, n[0] * n[1],
              n[1], 1};
  GemmArgs g2{n[0] * n[1], n[2], N[2], 1, y1, n[0] * n[1], 0, qt[2], n[2], 0, ctrl, n[2], 0, 0};
  hipError_t e = gemm<float, true>(g0, hs);
  if (e == hipSuccess) e = gemm<double, true>(g1, hs);
  if (e == hipSuccess) e = gemm<double, true>(g2, hs);
  return e;
}

// The spline on the sample grid, Fh = P x_0 B0 x_1 B1 x_2 B2, with the
// collocation tables bt[a] transposed (n_a x N_a); R1 is written transposed
// ([n2][N0 * N1]) for the same reason as Y1 above.
hipError_t run_recon(const int64_t N[3], const int64_t n[3], const double* ctrl,
                     const double* const bt[3], double* r0, double* r1, double* fh, hipStream_t hs) {
  GemmArgs g0{N[0], n[1] * n[2], n[0], 1, bt[0], N[0], 0, ctrl, n[1] * n[2], 0, r0, n[1] * n[2], 0, 0};
  GemmArgs g1{N[1], n[2], n[1], N[0], bt[1], N[1], 0, r0, n[2], n[1] * n[2], r1, N[0] * N[1], N[1], 1};
  GemmArgs g2{N[0] * N[1], N[2], n[2], 1, r1, N[0] * N[1], 0, bt[2], N[2], 0, fh, N[2], 0, 0};
  hipError_t e = gemm<double, true>(g0, hs);
  if (e == hipSuccess) e = gemm<double, true>(g1, hs);
  if (e == hipSuccess) e = gemm<double, true>(g2, hs);
  return e;
}

// ------------------------------------------------------------------ errors of a fit
constexpr int kErrRows = 512;     // rows per chunk of the column pass
constexpr int kMinMaxBlocks = 1024;

// Largest relative error |Fh - F| * inv_range of each grid row (i0, i1):
// one wave per row, lanes striding along axis 2.
__global__ __launch_bounds__(256) void err_rows_k(const double* __restrict__ fh,
                                                  const float* __restrict__ f, int64_t rows,
                                                  int64_t n2, double inv_range,
                                                  double* __restrict__ rowmax) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  double m = 0.0;
  for (int64_t c = lane; c < n2; c += 64)
    m = fmax(m, fabs(fh[row * n2 + c] - (double)f[row * n2 + c]) * inv_range);
#pragma unroll
  for (int o = 32; o; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) rowmax[row] = m;
}

// Largest relative error of each column i2 over chunks of kErrRows rows:
// colpart[chunk * n2 + c]; one thread per column of a chunk.
__global__ __launch_bounds__(256) void err_cols_k(const double* __restrict__ fh,
                                                  const float* __restrict__ f, int64_t rows,
                                                  int64_t n2, double inv_range,
                                                  double* __restrict__ colpart) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n2) return;
  const int64_t r0 = (int64_t)blockIdx.y * kErrRows, r1 = min(r0 + (int64_t)kErrRows, rows);
  double m = 0.0;
  for (int64_t r = r0; r < r1; ++r)
    m = fmax(m, fabs(fh[r * n2 + c] - (double)f[r * n2 + c]) * inv_range);
  colpart[blockIdx.y * n2 + c] = m;
}

// Per-workgroup (min, max) of the samples, for the data range.
__global__ __launch_bounds__(256) void minmax_k(const float* __restrict__ f, int64_t n,
                                                float2* __restrict__ part) {
  __shared__ float lo[256], hi[256];
  float a = __builtin_inff(), b = -__builtin_inff();
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
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

// Workspace layout (FP64): Q0, Q1, Q2 (B_a+ transposed), then Y0 = F x_0 B0+ (n0 x N1 x N2)
// and Y1 = Y0 x_1 B1+ (stored N2 x n0 x n1).
struct EncodeLayout {
  size_t q[3], y0, y1, total;
};

EncodeLayout encode_layout(const int32_t res[3], const int32_t n_ctrl[3]) {
  EncodeLayout L{};
  size_t o = 0;
  for (int a = 0; a < 3; ++a) {
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
    st = pseudo_inverse(T.data(), p, n, axis_u[a], N, a, Q[a]);
    if (st != MFA_OK) return st;
  }
  hipStream_t hs = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(work);
  for (int a = 0; a < 3; ++a) {
    hipError_t e = hipMemcpyAsync(wb + lay.q[a], Q[a].data(), Q[a].size() * sizeof(double),
                                  hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "encode: pseudo-inverse upload");
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
  const double* dq[3];
  for (int a = 0; a < 3; ++a) dq[a] = reinterpret_cast<const double*>(wb + lay.q[a]);
  double* y0 = reinterpret_cast<double*>(wb + lay.y0);
  double* y1 = reinterpret_cast<double*>(wb + lay.y1);
  const int64_t N0 = res[0], N1 = res[1], N2 = res[2];
  const int64_t n0 = n_ctrl[0], n1 = n_ctrl[1], n2 = n_ctrl[2];
  // tables dq[a] are B_a+ transposed: N_a x n_a
  const int64_t N[3] = {N0, N1, N2}, n[3] = {n0, n1, n2};
  hipError_t e = run_fit(N, n, values, ctrl, dq, y0, y1, hs);
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

// Workspace of the adaptive loop, sized for max_ctrl control points per axis.
struct AdaptLayout {
  size_t qt[3], bt[3], y0, y1, r0, r1, fh, rowmax, colpart, mm, total;
};

AdaptLayout adapt_layout(const int32_t res[3], const int32_t nm[3]) {
  AdaptLayout L{};
  const size_t N0 = res[0], N1 = res[1], N2 = res[2], m0 = nm[0], m1 = nm[1], m2 = nm[2];
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
  L.r1 = take(8 * m2 * N0 * N1);
  L.fh = take(8 * N0 * N1 * N2);
  L.rowmax = take(8 * N0 * N1);
  L.colpart = take(8 * ((N0 * N1 + kErrRows - 1) / kErrRows) * N2);
  L.mm = take(sizeof(float2) * kMinMaxBlocks);
  L.total = o;
  return L;
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
  const int64_t N[3] = {res[0], res[1], res[2]};
  const int64_t rows = N[0] * N[1], nchunk = (rows + kErrRows - 1) / kErrRows;
  if (nchunk > 65535) return fail(MFA_E_ARG, "res0 * res1 above %lld", 65535LL * kErrRows);
  // data range
  float2* mm = reinterpret_cast<float2*>(wb + lay.mm);
  hipLaunchKernelGGL(minmax_k, dim3(kMinMaxBlocks), dim3(256), 0, hs, values, rows * N[2], mm);
  std::vector<float2> hmm(kMinMaxBlocks);
  hipError_t e = hipMemcpyAsync(hmm.data(), mm, sizeof(float2) * kMinMaxBlocks, hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return hip_fail(e, "encode: data range");
  float lo = hmm[0].x, hi = hmm[0].y;
  for (const float2& v : hmm) {
    lo = std::min(lo, v.x);
    hi = std::max(hi, v.y);
  }
  const double range = (double)hi - (double)lo;
  const double inv_range = range > 0.0 ? 1.0 / range : 1.0;
  // initial knots: clamped uniform with n_init control points
  std::vector<double> T[3];
  for (int a = 0; a < 3; ++a) {
    T[a].resize(n_init[a] + degree[a] + 1);
    default_knots(n_init[a], degree[a], T[a].data());
  }
  std::vector<double> Q[3], Bt[3], rowmax(rows), colpart((size_t)nchunk * N[2]);
  int fits = 0;
  for (;;) {
    int64_t n[3];
    for (int a = 0; a < 3; ++a) n[a] = (int64_t)T[a].size() - degree[a] - 1;
    for (int a = 0; a < 3; ++a) {
      st = pseudo_inverse(T[a].data(), degree[a], (int)n[a], axis_u[a], res[a], a, Q[a], &Bt[a]);
      if (st != MFA_OK) return st;
      e = hipMemcpyAsync(at(lay.qt[a]), Q[a].data(), Q[a].size() * 8, hipMemcpyHostToDevice, hs);
      if (e == hipSuccess)
        e = hipMemcpyAsync(at(lay.bt[a]), Bt[a].data(), Bt[a].size() * 8, hipMemcpyHostToDevice, hs);
      if (e != hipSuccess) return hip_fail(e, "encode: table upload");
    }
    const double* qt[3] = {at(lay.qt[0]), at(lay.qt[1]), at(lay.qt[2])};
    const double* bt[3] = {at(lay.bt[0]), at(lay.bt[1]), at(lay.bt[2])};
    e = run_fit(N, n, values, ctrl, qt, at(lay.y0), at(lay.y1), hs);
    if (e == hipSuccess) e = run_recon(N, n, ctrl, bt, at(lay.r0), at(lay.r1), at(lay.fh), hs);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(err_rows_k, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, hs, at(lay.fh),
                         values, rows, N[2], inv_range, at(lay.rowmax));
      hipLaunchKernelGGL(err_cols_k, dim3((unsigned)((N[2] + 255) / 256), (unsigned)nchunk), dim3(256),
                         0, hs, at(lay.fh), values, rows, N[2], inv_range, at(lay.colpart));
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(rowmax.data(), at(lay.rowmax), rows * 8, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(colpart.data(), at(lay.colpart), colpart.size() * 8, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_fail(e, "encode: adaptive fit");
    // largest error per sample index of each axis
    std::vector<double> m[3];
    m[0].assign(N[0], 0.0);
    m[1].assign(N[1], 0.0);
    m[2].assign(N[2], 0.0);
    for (int64_t r = 0; r < rows; ++r) {
      m[0][r / N[1]] = std::max(m[0][r / N[1]], rowmax[r]);
      m[1][r % N[1]] = std::max(m[1][r % N[1]], rowmax[r]);
    }
    for (int64_t q = 0; q < nchunk; ++q)
      for (int64_t c = 0; c < N[2]; ++c) m[2][c] = std::max(m[2][c], colpart[q * N[2] + c]);
    double emax = 0.0;
    for (double v : m[0]) emax = std::max(emax, v);
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
