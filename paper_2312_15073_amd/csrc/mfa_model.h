// Host-side model record shared by the library's host sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "mfa.h"
#include "mfa_internal.h"

struct mfa_model_s {
  int device = 0;
  int degree = 0;
  mfa_dtype storage = MFA_F32;
  int grid[3] = {1, 1, 1};
  int nblocks = 1;
  double voxel = 0.0;
  std::vector<int32_t> n;       // 3 per block
  std::vector<int64_t> coff;    // element offset per block
  std::vector<int32_t> rs1;     // row stride per block
  int64_t n_ctrl_total = 0;
  std::vector<double> edges[3]; // block edges per axis (host copy), grid[a] + 1 each
  float vmin = 0.f, vmax = 0.f;
  void* d_ctrl = nullptr;
  int64_t ctrl_bytes = 0;
  mfa::SpanRec* d_rec = nullptr;
  float* d_mats = nullptr;
  mfa::DevBlock* d_blocks = nullptr;
  double* d_edges = nullptr;
  uint32_t* d_mcb = nullptr;
  uint32_t* d_scb[2] = {nullptr, nullptr};
  mfa::BucketWin* d_bwin = nullptr;
  mfa::SortBlk* d_sblk = nullptr;
  float* d_sedges = nullptr;
  int32_t* d_gtab = nullptr;
  int32_t* d_gmeta = nullptr;
  bool nonuniform = false;   // some axis has non-uniform knots (span guess tables)
  int64_t device_bytes = 0;
  int64_t n_buckets = 0;        // sort buckets (block, tile)
  void* d_ws = nullptr;         // scratch of sorted decodes, grown on demand
  size_t ws_bytes = 0;
  std::mutex ws_mu;             // guards d_ws and the fields below
  hipEvent_t ws_done = nullptr; // recorded after the last sorted call's kernels
  hipStream_t ws_stream = nullptr;
  bool ws_used = false;
  mfa::DevModel dm{};
};

// Error helpers: set the calling thread's last-error message and return st.
mfa_status fail(mfa_status st, const char* fmt, ...);
mfa_status hip_fail(hipError_t e, const char* what);
mfa::Storage storage_of(mfa_model m);
// Knot vectors: validation of a clamped nondecreasing vector on [0, 1]
// (n + p + 1 values; blk/axis only label the message) and the clamped
// uniform default T[p + j] = j / (n - p).
mfa_status check_knots(const double* T, int n, int p, int blk, int axis);
void default_knots(int n, int p, double* T);
mfa_status check_device(mfa_model m);
// Kernel family of a model (kKindPlain / kKindGraded / kKindMulti).  Only
// the single-block kernels have a variant with span guess tables; the
// serving kernel serves a model with a non-uniform axis through its
// multi-block form, whose exact span walk finds those spans.
inline int kernel_kind(mfa_model m) {
  return m->nblocks > 1 ? mfa::kKindMulti : (m->nonuniform ? mfa::kKindGraded : mfa::kKindPlain);
}
inline bool serve_multi(mfa_model m) { return m->nblocks > 1 || m->nonuniform; }
// Validated kernel arguments of a render of model m (shared by the direct
// entry point and the server); need_tf = false for the isosurface render,
// which uses neither the transfer function nor its value range.
mfa_status make_render_args(mfa_model m, const mfa_camera* cam, const mfa_render_params* rp,
                            int32_t w, int32_t h, float* rgba, const mfa_render_debug* dbg,
                            mfa::RenderArgs* out, bool need_tf = true);
