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
                          std::vector<double>& Q) {
  const int w = p + 1;
  std::vector<int> s(N);
  std::vector<double> Bv((size_t)N * w);
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
  // Y1 is written transposed, [N2][n0 * n1], so that the third product
  // reads its A operand along rows of 16 consecutive values
  GemmArgs g0{n0, N1 * N2, N0, 1, dq[0], n0, 0, values, N1 * N2, 0, y0, N1 * N2, 0, 0};
  GemmArgs g1{n1, N2, N1, n0, dq[1], n1, 0, y0, N2, N1 * N2, y1, n0 * n1, n1, 1};
  GemmArgs g2{n0 * n1, n2, N2, 1, y1, n0 * n1, 0, dq[2], n2, 0, ctrl, n2, 0, 0};
  hipError_t e = gemm<float, true>(g0, hs);
  if (e == hipSuccess) e = gemm<double, true>(g1, hs);
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
