// Serving loop: resident models, admission of render and point-query
// requests by a device-memory budget, batching of equal work items into
// persistent launches, completion and latency stamps.
//
// The paper re-runs its visualisation pipeline on every user change of
// transfer function, shading or view (Sec. IV-B); here many such requests
// from many clients share one GPU.  Requests are admitted first come first
// served while the bytes of their buffers fit the budget, split into work
// items (16x16 pixel tiles, 256-point chunks) and packed into batches of at
// most max_batch_items items, so a large frame spans several batches and
// small requests behind it still start soon.  Up to three batches run at
// once, each on its own stream as one persistent launch per model kind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "mfa.h"
#include "mfa_internal.h"
#include "mfa_model.h"

namespace mfa {
hipError_t launch_serve(int p, Storage s, bool multi, const DevModel* models, const ServeReq* reqs,
                        const ServeItem* items, int n_items, int* cursor, int grid, hipStream_t st);
}
using namespace mfa;

namespace {

constexpr int kTileEdge = 16;
constexpr int kChunk = 256;
constexpr int kMaxInFlight = 3;

struct Req {
  uint64_t ticket = 0;
  int model = 0;
  ServeReq desc{};
  int64_t bytes = 0;
  int n_items = 0;
  int next_item = 0;        // first item not yet placed in a batch
  int items_left = 0;       // items not yet completed
  bool admitted = false;
  bool done = false;
  int status = MFA_OK;
  double t_submit = 0, t_admit = -1, t_start = -1, t_done = -1;
};

struct Variant {
  int p;
  Storage s;
  bool multi;
  bool operator<(const Variant& o) const {
    return std::tie(p, s, multi) < std::tie(o.p, o.s, o.multi);
  }
};

struct Batch {
  int slot = 0;
  int seq = 0;              // launch number, 1-based
  int status = MFA_OK;      // MFA_E_DEVICE when its launch or its kernels failed
  hipEvent_t ev = nullptr;
  double t_launch = 0, t_end_fake = 0;
  std::vector<std::pair<Req*, int>> parts;   // request, items of it in this batch
};

// Device and pinned host buffers of one batch slot.
struct Slot {
  uint8_t* d_buf = nullptr;     // cursors | requests | items of one batch
  uint8_t* h_stage = nullptr;   // pinned staging of d_buf
  hipStream_t stream = nullptr; // batches of different slots overlap
};

}  // namespace

struct mfa_server_s {
  mfa_server_config cfg{};
  bool fake = false;
  int device = -1;
  int cus = 0;
  std::vector<mfa_model> models;
  DevModel* d_models = nullptr;
  int d_models_cap = 0;
  int max_reqs = 0;
  Slot slots[kMaxInFlight];
  bool slot_busy[kMaxInFlight] = {false, false, false};

  // mu guards the queue, the requests and their stats (clients and the
  // scheduler); launch_mu serialises device-side changes of the model
  // table against batch launches, which run outside mu so that submit and
  // poll never wait for a launch.  Order: launch_mu before mu.
  std::mutex mu;
  std::mutex launch_mu;
  std::condition_variable cv;       // scheduler wake-up
  std::condition_variable cv_done;  // request completions
  std::deque<Req*> queue;           // requests with items not yet batched
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<Batch> inflight;
  int64_t in_use = 0;
  uint64_t next_ticket = 1;
  int next_seq = 1;
  bool stop = false;
  std::thread th;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double fake_busy_until = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void run();
  bool form_batch(Batch& b, std::vector<ServeItem>& items, std::vector<ServeReq>& descs,
                  std::vector<std::pair<Variant, std::pair<int, int>>>& ranges);
  void retire(Batch& b, double t);
  mfa_status launch(Batch& b, const std::vector<ServeItem>& items, const std::vector<ServeReq>& descs,
                    const std::vector<std::pair<Variant, std::pair<int, int>>>& ranges);
};

static Variant variant_of(mfa_model m) {
  if (!m) return Variant{3, Storage::F32, false};
  return Variant{m->degree, storage_of(m), serve_multi(m)};
}

// Places the next items of the queued requests, first come first served,
// into a batch; admits requests while their bytes fit the budget.
bool mfa_server_s::form_batch(Batch& b, std::vector<ServeItem>& items, std::vector<ServeReq>& descs,
                              std::vector<std::pair<Variant, std::pair<int, int>>>& ranges) {
  const int cap = cfg.max_batch_items;
  std::vector<std::pair<Variant, ServeItem>> tmp;
  const double t = now();
  while (!queue.empty() && (int)tmp.size() < cap && (int)b.parts.size() < max_reqs) {
    Req* r = queue.front();
    if (!r->admitted) {
      if (in_use + r->bytes > cfg.hbm_budget_bytes) break;   // wait for memory, keep order
      r->admitted = true;
      in_use += r->bytes;
      r->t_admit = t;
    }
    const int take = std::min(r->n_items - r->next_item, cap - (int)tmp.size());
    const int slot_req = (int)b.parts.size();
    const Variant v = variant_of(models[r->model]);
    for (int q = 0; q < take; ++q) tmp.push_back({v, ServeItem{slot_req, r->next_item + q}});
    descs.push_back(r->desc);
    b.parts.push_back({r, take});
    r->next_item += take;
    if (r->next_item == r->n_items) queue.pop_front();
  }
  if (tmp.empty()) return false;
  // group items by kernel kind, keeping arrival order inside each kind
  std::stable_sort(tmp.begin(), tmp.end(),
                   [](const auto& a, const auto& c) { return a.first < c.first; });
  for (size_t q = 0; q < tmp.size();) {
    size_t e = q;
    while (e < tmp.size() && !(tmp[q].first < tmp[e].first) && !(tmp[e].first < tmp[q].first)) ++e;
    ranges.push_back({tmp[q].first, {(int)q, (int)e}});
    q = e;
  }
  for (auto& x : tmp) items.push_back(x.second);
  return true;
}

// Stages and enqueues one batch; runs on the scheduler thread without mu
// (it touches only the batch, its slot and the model table, under
// launch_mu).  The fake executor models the batch's duration instead and
// fails the batch numbered cfg.fake_fail_batch.
mfa_status mfa_server_s::launch(Batch& b, const std::vector<ServeItem>& items,
                                const std::vector<ServeReq>& descs,
                                const std::vector<std::pair<Variant, std::pair<int, int>>>& ranges) {
  if (fake) {
    const double start = std::max(b.t_launch, fake_busy_until);
    b.t_end_fake = start + 1e-6 * cfg.fake_item_us * (double)items.size();
    fake_busy_until = b.t_end_fake;
    if (b.seq == cfg.fake_fail_batch) return fail(MFA_E_DEVICE, "injected failure of batch %d", b.seq);
    return MFA_OK;
  }
  Slot& S = slots[b.slot];
  // one packed copy per batch: cursors (zeroed) | requests | items
  const size_t o_req = 64 * sizeof(int);
  const size_t o_item = (o_req + descs.size() * sizeof(ServeReq) + 15) & ~(size_t)15;
  const size_t total = o_item + items.size() * sizeof(ServeItem);
  std::memset(S.h_stage, 0, o_req);
  std::memcpy(S.h_stage + o_req, descs.data(), descs.size() * sizeof(ServeReq));
  std::memcpy(S.h_stage + o_item, items.data(), items.size() * sizeof(ServeItem));
  hipError_t e = hipMemcpyAsync(S.d_buf, S.h_stage, total, hipMemcpyHostToDevice, S.stream);
  int* d_cursors = (int*)S.d_buf;
  const ServeReq* d_reqs = (const ServeReq*)(S.d_buf + o_req);
  const ServeItem* d_items = (const ServeItem*)(S.d_buf + o_item);
  for (size_t k = 0; k < ranges.size() && e == hipSuccess; ++k) {
    const Variant& v = ranges[k].first;
    const int a = ranges[k].second.first, n = ranges[k].second.second - a;
    const int grid = std::min(n, 4 * cus);
    e = launch_serve(v.p, v.s, v.multi, d_models, d_reqs, d_items + a, n, d_cursors + k, grid,
                     S.stream);
  }
  if (e == hipSuccess) e = hipEventRecord(b.ev, S.stream);
  if (e != hipSuccess) return hip_fail(e, "server batch launch");
  return MFA_OK;
}

// A failed batch fails every request with items in it (a request spanning
// batches takes the first failure); each request releases its budget when
// its last item is retired, failed or not.
void mfa_server_s::retire(Batch& b, double t) {
  for (auto& pr : b.parts) {
    Req* r = pr.first;
    r->items_left -= pr.second;
    if (b.status != MFA_OK && r->status == MFA_OK) r->status = b.status;
    if (r->items_left == 0) {
      r->done = true;
      r->t_done = t;
      in_use -= r->bytes;
    }
  }
  slot_busy[b.slot] = false;
  if (b.ev) (void)hipEventDestroy(b.ev);
  b.ev = nullptr;
  cv_done.notify_all();
}

void mfa_server_s::run() {
  if (!fake) (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // retire finished batches (slots run on separate streams, so in any order)
    for (auto it = inflight.begin(); it != inflight.end();) {
      bool fin;
      if (fake) {
        fin = now() >= it->t_end_fake;
      } else {
        const hipError_t q = it->ev ? hipEventQuery(it->ev) : hipSuccess;
        if (q != hipSuccess && q != hipErrorNotReady) it->status = MFA_E_DEVICE;
        fin = q != hipErrorNotReady;
      }
      if (fin) {
        retire(*it, now());
        it = inflight.erase(it);
      } else {
        ++it;
      }
    }
    if (stop && queue.empty() && inflight.empty()) return;
    // start a batch when a slot is free
    if ((int)inflight.size() < kMaxInFlight && !queue.empty()) {
      int slot = 0;
      while (slot_busy[slot]) ++slot;
      Batch b;
      b.slot = slot;
      std::vector<ServeItem> items;
      std::vector<ServeReq> descs;
      std::vector<std::pair<Variant, std::pair<int, int>>> ranges;
      if (form_batch(b, items, descs, ranges)) {
        slot_busy[slot] = true;
        b.seq = next_seq++;
        b.t_launch = now();
        for (auto& pr : b.parts)
          if (pr.first->t_start < 0) pr.first->t_start = b.t_launch;
        // the launch (staging copy, kernels, event) runs without mu
        lk.unlock();
        mfa_status st = MFA_OK;
        {
          std::lock_guard<std::mutex> lg(launch_mu);
          if (!fake) {
            const hipError_t e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
            if (e != hipSuccess) {
              b.ev = nullptr;
              st = hip_fail(e, "server batch event");
            }
          }
          if (st == MFA_OK) st = launch(b, items, descs, ranges);
        }
        lk.lock();
        if (st != MFA_OK) {
          // the batch failed before (all of) its work was enqueued: its
          // event, if recorded at all, is not waited for
          b.status = MFA_E_DEVICE;
          // work of it that was enqueued still reads the slot's buffers:
          // the slot is free again only once its stream has passed it
          if (!fake) (void)hipStreamSynchronize(slots[b.slot].stream);
          if (b.ev) (void)hipEventDestroy(b.ev);
          b.ev = nullptr;
          b.t_end_fake = now();
        }
        inflight.push_back(std::move(b));
        continue;
      }
    }
    // nothing to start: wait for a submission or poll the running batches
    if (inflight.empty())
      cv.wait(lk, [&] { return stop || !queue.empty(); });
    else
      cv.wait_for(lk, std::chrono::microseconds(20));
  }
}

static mfa_status server_free(mfa_server s) {
  if (!s) return MFA_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  if (!s->fake) {
    for (auto& b : s->inflight)
      if (b.ev) (void)hipEventDestroy(b.ev);
    for (auto& S : s->slots) {
      if (S.d_buf) (void)hipFree(S.d_buf);
      if (S.h_stage) (void)hipHostFree(S.h_stage);
      if (S.stream) (void)hipStreamDestroy(S.stream);
    }
    if (s->d_models) (void)hipFree(s->d_models);
  }
  delete s;
  return MFA_OK;
}

extern "C" mfa_status mfa_server_create(const mfa_server_config* cfg, mfa_server* out) {
  if (!cfg || !out) return fail(MFA_E_ARG, "null argument");
  *out = nullptr;
  if (cfg->hbm_budget_bytes <= 0) return fail(MFA_E_ARG, "hbm_budget_bytes must be > 0");
  if (cfg->queue_cap <= 0) return fail(MFA_E_ARG, "queue_cap must be > 0");
  if (cfg->max_batch_items < 0 || cfg->max_batch_items > (1 << 22))
    return fail(MFA_E_ARG, "max_batch_items out of range");
  if (cfg->flags & ~MFA_SERVER_FAKE_EXECUTOR) return fail(MFA_E_ARG, "unknown flags");
  const bool fake = (cfg->flags & MFA_SERVER_FAKE_EXECUTOR) != 0;
  if (fake && !(cfg->fake_item_us >= 0.0)) return fail(MFA_E_ARG, "fake_item_us must be >= 0");
  mfa_server s = new mfa_server_s();
  s->cfg = *cfg;
  if (s->cfg.max_batch_items == 0) s->cfg.max_batch_items = 8192;
  s->fake = fake;
  s->max_reqs = std::min(s->cfg.queue_cap, 4096);
  if (!fake) {
    hipError_t e = hipGetDevice(&s->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, s->device);
    if (e == hipSuccess) s->cus = prop.multiProcessorCount;
    for (auto& S : s->slots) {
      const size_t bytes = 64 * sizeof(int) + (size_t)s->max_reqs * sizeof(ServeReq) + 16 +
                           (size_t)s->cfg.max_batch_items * sizeof(ServeItem);
      if (e == hipSuccess) e = hipMalloc((void**)&S.d_buf, bytes);
      if (e == hipSuccess) e = hipHostMalloc((void**)&S.h_stage, bytes, hipHostMallocDefault);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking);
    }
    if (e != hipSuccess) {
      server_free(s);
      return hip_fail(e, "server resources");
    }
  }
  s->th = std::thread([s] { s->run(); });
  *out = s;
  return MFA_OK;
}

extern "C" mfa_status mfa_server_add_model(mfa_server s, mfa_model m, int32_t* model_id) {
  if (!s || !model_id) return fail(MFA_E_ARG, "null argument");
  if (!m && !s->fake) return fail(MFA_E_ARG, "null model");
  if (m && !s->fake && m->device != s->device)
    return fail(MFA_E_ARG, "model on device %d, server on device %d", m->device, s->device);
  std::lock_guard<std::mutex> lg(s->launch_mu);    // no batch is being launched
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->fake) {
    // grow the device model table; requests in flight keep using the old
    // one until the stream has passed them, so wait for the stream first
    const int n = (int)s->models.size() + 1;
    if (n > s->d_models_cap) {
      const int cap = std::max(8, 2 * n);
      DevModel* nd = nullptr;
      hipError_t e = hipSuccess;
      for (auto& S : s->slots)
        if (e == hipSuccess && S.stream) e = hipStreamSynchronize(S.stream);
      if (e == hipSuccess) e = hipMalloc((void**)&nd, (size_t)cap * sizeof(DevModel));
      if (e == hipSuccess && s->d_models)
        e = hipMemcpy(nd, s->d_models, (size_t)(n - 1) * sizeof(DevModel), hipMemcpyDeviceToDevice);
      if (e != hipSuccess) return hip_fail(e, "server model table");
      if (s->d_models) (void)hipFree(s->d_models);
      s->d_models = nd;
      s->d_models_cap = cap;
    }
    hipError_t e = hipMemcpy(s->d_models + (n - 1), &m->dm, sizeof(DevModel), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "server model table");
  }
  s->models.push_back(m);
  *model_id = (int32_t)s->models.size() - 1;
  return MFA_OK;
}

extern "C" mfa_status mfa_server_submit(mfa_server s, const mfa_request* rq, uint64_t* ticket) {
  if (!s || !rq || !ticket) return fail(MFA_E_ARG, "null argument");
  std::unique_ptr<Req> r(new Req());
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (rq->model_id < 0 || rq->model_id >= (int)s->models.size())
      return fail(MFA_E_ARG, "unknown model id %d", rq->model_id);
  }
  mfa_model m = s->models[rq->model_id];
  r->model = rq->model_id;
  r->desc.model = rq->model_id;
  if (rq->kind == MFA_REQ_RENDER) {
    if (m) {
      mfa_status st = make_render_args(m, &rq->camera, &rq->params, rq->w, rq->h, rq->rgba, nullptr,
                                       &r->desc.ra);
      if (st != MFA_OK) return st;
    } else if (!rq->rgba || rq->w < 1 || rq->h < 1 || rq->w > 16384 || rq->h > 16384) {
      return fail(MFA_E_ARG, "bad render request");
    } else {
      r->desc.ra.w = rq->w;
      r->desc.ra.h = rq->h;
    }
    r->desc.kind = kServeRender;
    r->n_items = ((rq->w + kTileEdge - 1) / kTileEdge) * ((rq->h + kTileEdge - 1) / kTileEdge);
    r->bytes = (int64_t)rq->w * rq->h * 16 + 256 * 16;
  } else if (rq->kind == MFA_REQ_POINTS) {
    if (rq->n < 1 || rq->n >= (1ll << 31)) return fail(MFA_E_ARG, "n out of range");
    if (!rq->xyz || !rq->out) return fail(MFA_E_ARG, "null xyz/out");
    r->desc.kind = kServePoints;
    r->desc.xyz = rq->xyz;
    r->desc.out = rq->out;
    r->desc.n = rq->n;
    r->n_items = (int)((rq->n + kChunk - 1) / kChunk);
    r->bytes = rq->n * 28;
  } else {
    return fail(MFA_E_ARG, "unknown request kind %d", rq->kind);
  }
  r->items_left = r->n_items;
  std::lock_guard<std::mutex> g(s->mu);
  if (r->bytes > s->cfg.hbm_budget_bytes)
    return fail(MFA_E_BUDGET, "request needs %lld bytes, budget %lld", (long long)r->bytes,
                (long long)s->cfg.hbm_budget_bytes);
  if ((int)s->queue.size() >= s->cfg.queue_cap) return fail(MFA_E_BUSY, "queue full");
  if (s->stop) return fail(MFA_E_ARG, "server stopping");
  r->ticket = s->next_ticket++;
  r->t_submit = s->now();
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->ticket, std::move(r));
  s->cv.notify_one();
  return MFA_OK;
}

static void fill_stats(const Req& r, mfa_request_stats* st) {
  st->t_submit = r.t_submit;
  st->t_admit = r.t_admit;
  st->t_start = r.t_start;
  st->t_done = r.t_done;
  st->status = r.status;
  st->done = r.done ? 1 : 0;
}

extern "C" mfa_status mfa_server_poll(mfa_server s, uint64_t ticket, mfa_request_stats* st) {
  if (!s || !st) return fail(MFA_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MFA_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  fill_stats(*it->second, st);
  return MFA_OK;
}

extern "C" mfa_status mfa_server_wait(mfa_server s, uint64_t ticket, mfa_request_stats* st) {
  if (!s || !st) return fail(MFA_E_ARG, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MFA_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->done; });
  fill_stats(*r, st);
  return r->status == MFA_OK ? MFA_OK : fail((mfa_status)r->status, "request failed on the device");
}

extern "C" mfa_status mfa_server_release(mfa_server s, uint64_t ticket) {
  if (!s) return fail(MFA_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MFA_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (!it->second->done) return fail(MFA_E_ARG, "ticket %llu still running", (unsigned long long)ticket);
  s->reqs.erase(it);
  return MFA_OK;
}

extern "C" mfa_status mfa_server_destroy(mfa_server s) { return server_free(s); }
