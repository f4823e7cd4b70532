// Serving engine: continuous batching of scoring requests on one GPU.
//
// The paper's screening jobs push batches of poses through the model on each
// GPU and collect identifiers and predictions (Sec. 4.2); this engine is the
// request-driven form of that loop.  Requests (one or more poses each, each with
// its own grid size) are copied at submission and queued.  A host scheduler
// thread owns `n_slots` device slots -- one stream, one scoring context with
// resident weights and scratch, pinned staging buffers -- and whenever a slot is
// free it packs queued requests of one grid size into a batch (continuous
// batching: work that arrives while other batches run is admitted as slots free
// up, and batches on different slots overlap on the device).  A batch is padded
// with empty poses to a power-of-two bucket so its kernel sequence can be
// captured once per (grid size, bucket) as a hipGraph and replayed.  Scores do
// not depend on the batch a pose lands in: every kernel computes each pose
// independently and in a fixed order.  Hence a batch whose device checks fail is
// scored again one request at a time, so that only the request at fault reports
// the error and every other request still gets the scores it would get alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cf_internal.h"
#include "cf_queue.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  int n_poses = 0, G = 0;
  std::vector<int32_t> off, xyz;
  std::vector<float> feat;
  std::vector<uint8_t> lig;
  Clock::time_point t_submit;
  std::vector<float> scores;
  int status = CF_OK;
  bool done = false;
  double latency_ms = 0.0;
  int64_t atoms() const { return off[n_poses]; }
};

struct Slot {
  cf_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  int32_t *h_off = nullptr, *h_xyz = nullptr;
  float *h_feat = nullptr, *h_scores = nullptr;
  uint8_t *h_lig = nullptr;
  int32_t *d_off = nullptr, *d_xyz = nullptr;
  float *d_feat = nullptr, *d_scores = nullptr;
  uint8_t *d_lig = nullptr;
  bool busy = false;
  std::vector<std::pair<Request *, int>> members;  // request, first pose in the batch
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  int64_t graphs_gen = -1;  // scratch generation of the context the graphs were captured against
};

// Captured graphs hold the context's scratch pointers; once the context has
// reallocated any scratch buffer they must be dropped (and captured again).
void drop_stale_graphs(Slot &s) {
  const int64_t gen = cf::scratch_generation(s.ctx);
  if (gen == s.graphs_gen) return;
  for (auto &kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
  s.graphs.clear();
  s.graphs_gen = gen;
}

}  // namespace

struct cf_engine {
  cf_engine_config cfg{};
  int device = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  cf::RequestQueue<Request> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1;
  std::thread worker;
  std::atomic<bool> stop{false};
  std::atomic<int64_t> poses_done{0}, batches{0}, replays{0}, in_flight{0};
  std::string last_error;
};

namespace {

int bucket_for(int n, int cap) {
  int b = 16;
  while (b < n) b <<= 1;
  return b < cap ? b : cap;
}

void free_slot(Slot &s) {
  for (auto &kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
  if (s.ev) (void)hipEventDestroy(s.ev);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  void *hp[] = {s.h_off, s.h_xyz, s.h_feat, s.h_scores, s.h_lig};
  for (void *p : hp)
    if (p) (void)hipHostFree(p);
  void *dp[] = {s.d_off, s.d_xyz, s.d_feat, s.d_scores, s.d_lig};
  for (void *p : dp)
    if (p) (void)hipFree(p);
  if (s.ctx) cf_destroy(s.ctx);
}

// Pack requests into the slot's pinned staging (pose rows in request order,
// padded with empty poses up to `bucket`) and copy them to the slot's device
// buffers on its stream.  Returns the number of real poses in *np_out.
int stage_requests(cf_engine *e, Slot &s, const std::vector<Request *> &take, int bucket_cap, int *np_out,
                   int *bucket_out, int64_t *na_out) {
  int np = 0;
  int64_t na = 0;
  s.members.clear();
  s.h_off[0] = 0;
  for (Request *r : take) {
    s.members.push_back({r, np});
    const int64_t ra = r->atoms();
    memcpy(s.h_xyz + 3 * na, r->xyz.data(), sizeof(int32_t) * 3 * ra);
    memcpy(s.h_feat + (size_t)CF_NCH * na, r->feat.data(), sizeof(float) * CF_NCH * ra);
    memcpy(s.h_lig + na, r->lig.data(), ra);
    for (int p = 0; p < r->n_poses; ++p) s.h_off[np + p + 1] = (int32_t)(na + r->off[p + 1]);
    np += r->n_poses;
    na += ra;
  }
  const int bucket = bucket_cap > 0 ? bucket_for(np, bucket_cap) : np;
  for (int p = np; p < bucket; ++p) s.h_off[p + 1] = (int32_t)na;  // empty padding poses
  hipStream_t st = s.stream;
  if (hipMemcpyAsync(s.d_off, s.h_off, sizeof(int32_t) * (bucket + 1), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s.d_xyz, s.h_xyz, sizeof(int32_t) * 3 * na, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s.d_feat, s.h_feat, sizeof(float) * CF_NCH * na, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s.d_lig, s.h_lig, na, hipMemcpyHostToDevice, st)) {
    e->last_error = "engine H2D copy failed";
    return CF_ERR_HIP;
  }
  *np_out = np;
  *bucket_out = bucket;
  *na_out = na;
  return CF_OK;
}

// Launch one packed batch on a free slot.  Called by the worker with mu held.
int launch_batch(cf_engine *e, Slot &s, std::vector<Request *> &take, int G) {
  const int cap_p = e->cfg.slot_poses;
  int np = 0, bucket = 0;
  int64_t na = 0;
  int rc = stage_requests(e, s, take, cap_p, &np, &bucket, &na);
  if (rc) return rc;
  hipStream_t st = s.stream;
  // The batch descriptor uses the slot's capacity as n_atoms: buffers hold that
  // many rows, and fixed arguments let one captured graph serve every batch of
  // this (G, bucket).
  cf_pose_batch b{};
  b.n_poses = bucket;
  b.n_atoms = (int32_t)std::min<int64_t>(e->cfg.slot_atoms, (int64_t)bucket * CF_MAX_POSE_ATOMS);
  b.atom_off = s.d_off;
  b.xyz = s.d_xyz;
  b.feat = s.d_feat;
  b.is_lig = s.d_lig;
  b.center = nullptr;
  if (e->cfg.use_graphs) {
    auto key = std::make_pair(G, bucket);
    drop_stale_graphs(s);
    auto it = s.graphs.find(key);
    if (it == s.graphs.end()) {
      // warm-up (allocates scratch, outside capture), then capture
      if ((rc = cf_score_poses(s.ctx, &b, G, s.d_scores, st))) return rc;
      drop_stale_graphs(s);  // the warm-up may have grown scratch other graphs point into
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) return CF_ERR_HIP;
      rc = cf_score_poses(s.ctx, &b, G, s.d_scores, st);
      const hipError_t ce = hipStreamEndCapture(st, &g);
      if (rc || ce != hipSuccess) return rc ? rc : CF_ERR_HIP;
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return CF_ERR_HIP;
      }
      (void)hipGraphDestroy(g);
      it = s.graphs.emplace(key, ex).first;
    }
    if (hipGraphLaunch(it->second, st) != hipSuccess) return CF_ERR_HIP;
    e->replays++;
  } else {
    if ((rc = cf_score_poses(s.ctx, &b, G, s.d_scores, st))) return rc;
  }
  if (hipMemcpyAsync(s.h_scores, s.d_scores, sizeof(float) * np, hipMemcpyDeviceToHost, st) ||
      hipEventRecord(s.ev, st))
    return CF_ERR_HIP;
  s.busy = true;
  e->batches++;
  e->in_flight += np;
  return CF_OK;
}

// Score one request alone on the slot (eager launches, synchronous) and return
// its status; its scores go to r->scores.
int score_alone(cf_engine *e, Slot &s, Request *r) {
  int np = 0, bucket = 0;
  int64_t na = 0;
  int rc = stage_requests(e, s, std::vector<Request *>{r}, 0, &np, &bucket, &na);
  if (rc == CF_OK) {
    cf_pose_batch b{};
    b.n_poses = np;
    b.n_atoms = (int32_t)na;
    b.atom_off = s.d_off;
    b.xyz = s.d_xyz;
    b.feat = s.d_feat;
    b.is_lig = s.d_lig;
    rc = cf_score_poses(s.ctx, &b, r->G, s.d_scores, s.stream);
  }
  if (rc == CF_OK && hipMemcpyAsync(s.h_scores, s.d_scores, sizeof(float) * np, hipMemcpyDeviceToHost, s.stream))
    rc = CF_ERR_HIP;
  const int st = cf_stream_status(s.ctx, s.stream, nullptr, nullptr);
  if (rc == CF_OK) rc = st;
  r->scores.assign(s.h_scores, s.h_scores + r->n_poses);
  return rc;
}

void finish_slot(cf_engine *e, Slot &s) {
  int64_t need_c = 0, need_n = 0;
  const int st = cf_stream_status(s.ctx, s.stream, &need_c, &need_n);
  if (st != CF_OK) e->last_error = std::string("device status: ") + cf_last_error();
  const auto members = s.members;  // score_alone restages the slot
  int np = 0;
  for (auto &m : members) {
    Request *r = m.first;
    r->scores.assign(s.h_scores + m.second, s.h_scores + m.second + r->n_poses);
    r->status = st;
    np += r->n_poses;
  }
  // A device-detected error (e.g. one pose's neighbour lists overflowing the
  // batch's edge capacity) is reported for the whole batch: score each request
  // alone to find which one is at fault.  The others' scores equal what the batch
  // would have given them (scores never depend on the batch).
  if (st != CF_OK && members.size() > 1)
    for (auto &m : members) m.first->status = score_alone(e, s, m.first);
  const auto now = Clock::now();
  for (auto &m : members) {
    Request *r = m.first;
    r->latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    r->done = true;
  }
  e->poses_done += np;
  e->in_flight -= np;
  s.members.clear();
  s.busy = false;
}

void worker_main(cf_engine *e) {
  (void)hipSetDevice(e->device);
  std::unique_lock<std::mutex> lk(e->mu);
  while (!e->stop) {
    bool progressed = false;
    for (Slot &s : e->slots)
      if (s.busy && hipEventQuery(s.ev) == hipSuccess) {
        finish_slot(e, s);
        progressed = true;
      }
    for (Slot &s : e->slots) {
      if (s.busy || e->pending.empty()) continue;
      // pack queued requests with the head's grid size, in arrival order
      std::vector<Request *> take = e->pending.take_batch(e->cfg.slot_poses, e->cfg.slot_atoms);
      const int G = take.front()->G;
      const int rc = launch_batch(e, s, take, G);
      if (rc != CF_OK) {
        e->last_error = std::string("batch launch failed: ") + cf_last_error();
        for (Request *r : take) {
          r->status = rc;
          r->done = true;
        }
        s.busy = false;
        (void)hipStreamSynchronize(s.stream);
      }
      progressed = true;
    }
    e->cv.notify_all();
    if (!progressed) {
      bool any_busy = false;
      for (Slot &s : e->slots) any_busy |= s.busy;
      // idle: sleep until work arrives; busy: poll the slots' events
      if (any_busy)
        e->cv.wait_for(lk, std::chrono::microseconds(20));
      else
        e->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

int efail(cf_engine *e, int code, const char *msg) {
  if (e) e->last_error = msg;
  return code;
}

}  // namespace

extern "C" {

int cf_engine_create(const void *blob, size_t nbytes, int precision, const cf_engine_config *cfg, cf_engine **out) {
  if (!out || !cfg) return CF_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 8 || cfg->slot_poses < 1 || cfg->slot_poses > 512 || cfg->slot_atoms < 1 ||
      cfg->slot_atoms > (int64_t)cfg->slot_poses * CF_MAX_POSE_ATOMS || cfg->slot_atoms > INT32_MAX)
    return CF_ERR_INVALID_ARG;
  auto e = std::make_unique<cf_engine>();
  e->cfg = *cfg;
  if (hipGetDevice(&e->device) != hipSuccess) return CF_ERR_HIP;
  const int64_t budget = cfg->hbm_budget_bytes > 0 ? cfg->hbm_budget_bytes : ((int64_t)32 << 30);
  const int64_t per_slot = budget / cfg->n_slots;
  e->slots.resize(cfg->n_slots);
  const size_t A = (size_t)cfg->slot_atoms, P = (size_t)cfg->slot_poses;
  for (Slot &s : e->slots) {
    int rc = cf_create(blob, nbytes, precision, per_slot, &s.ctx);
    if (rc) {
      for (Slot &t : e->slots) free_slot(t);
      return rc;
    }
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) ||
        hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) ||
        hipHostMalloc((void **)&s.h_off, sizeof(int32_t) * (P + 1), 0) ||
        hipHostMalloc((void **)&s.h_xyz, sizeof(int32_t) * 3 * A, 0) ||
        hipHostMalloc((void **)&s.h_feat, sizeof(float) * CF_NCH * A, 0) ||
        hipHostMalloc((void **)&s.h_lig, A, 0) || hipHostMalloc((void **)&s.h_scores, sizeof(float) * P, 0) ||
        hipMalloc(&s.d_off, sizeof(int32_t) * (P + 1)) || hipMalloc(&s.d_xyz, sizeof(int32_t) * 3 * A) ||
        hipMalloc(&s.d_feat, sizeof(float) * CF_NCH * A) || hipMalloc(&s.d_lig, A) ||
        hipMalloc(&s.d_scores, sizeof(float) * P)) {
      for (Slot &t : e->slots) free_slot(t);
      return CF_ERR_OOM;
    }
  }
  cf_engine *raw = e.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return CF_OK;
}

int cf_engine_submit(cf_engine *e, int32_t n_poses, const int32_t *atom_off, const int32_t *xyz, const float *feat,
                     const uint8_t *is_lig, int32_t G, uint64_t *ticket) {
  if (!e || !ticket || !atom_off || !xyz || !feat || !is_lig) return efail(e, CF_ERR_INVALID_ARG, "null argument");
  if (n_poses < 1 || n_poses > e->cfg.slot_poses) return efail(e, CF_ERR_INVALID_ARG, "n_poses outside 1..slot_poses");
  if (G < 8 || G > 96 || (G & 3)) return efail(e, CF_ERR_UNSUPPORTED, "grid size must be a multiple of 4 in 8..96");
  if (atom_off[0] != 0) return efail(e, CF_ERR_INVALID_ARG, "atom_off[0] must be 0");
  for (int p = 0; p < n_poses; ++p) {
    const int32_t d = atom_off[p + 1] - atom_off[p];
    if (d < 1 || d > CF_MAX_POSE_ATOMS) return efail(e, CF_ERR_INVALID_ARG, "each pose needs 1..4096 atoms");
  }
  const int64_t na = atom_off[n_poses];
  if (na > e->cfg.slot_atoms) return efail(e, CF_ERR_INVALID_ARG, "request has more atoms than a slot holds");
  // the device checks the same bound, but for a whole batch: reject a bad
  // request here so that it never shares a batch with others
  for (int64_t i = 0; i < (int64_t)CF_NCH * na; ++i)
    if (!(std::fabs(feat[i]) <= cf::kFeatMax))
      return efail(e, CF_ERR_INVALID_ARG, "feature value not finite or |value| > 64");
  auto r = std::make_unique<Request>();
  r->n_poses = n_poses;
  r->G = G;
  r->off.assign(atom_off, atom_off + n_poses + 1);
  r->xyz.assign(xyz, xyz + 3 * na);
  r->feat.assign(feat, feat + (size_t)CF_NCH * na);
  r->lig.assign(is_lig, is_lig + na);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(e->mu);
    r->id = e->next_id++;
    *ticket = r->id;
    e->pending.push(r.get());
    e->reqs.emplace(r->id, std::move(r));
  }
  e->cv.notify_all();
  return CF_OK;
}

int cf_engine_poll(cf_engine *e, uint64_t ticket, float *scores_out, int32_t *done, double *latency_ms) {
  if (!e || !done) return efail(e, CF_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(e->mu);
  auto it = e->reqs.find(ticket);
  if (it == e->reqs.end()) return efail(e, CF_ERR_INVALID_ARG, "unknown ticket");
  Request *r = it->second.get();
  *done = r->done ? 1 : 0;
  if (!r->done) return CF_OK;
  if (r->status == CF_ERR_CANCELLED) {
    e->reqs.erase(it);
    return efail(e, CF_ERR_CANCELLED, "request was cancelled");
  }
  if (scores_out) memcpy(scores_out, r->scores.data(), sizeof(float) * r->scores.size());
  if (latency_ms) *latency_ms = r->latency_ms;
  const int st = r->status;
  e->reqs.erase(it);
  return st;
}

int cf_engine_cancel(cf_engine *e, uint64_t ticket, int32_t *cancelled) {
  if (!e || !cancelled) return efail(e, CF_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(e->mu);
  *cancelled = 0;
  auto it = e->reqs.find(ticket);
  if (it == e->reqs.end()) return efail(e, CF_ERR_INVALID_ARG, "unknown ticket");
  Request *r = it->second.get();
  if (!r->done && e->pending.cancel(r)) {
    r->status = CF_ERR_CANCELLED;
    r->done = true;
    *cancelled = 1;
  }
  e->cv.notify_all();
  return CF_OK;
}

int cf_engine_wait_all(cf_engine *e) {
  if (!e) return CF_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] {
    if (!e->pending.empty()) return false;
    for (Slot &s : e->slots)
      if (s.busy) return false;
    return true;
  });
  return CF_OK;
}

int cf_engine_info(cf_engine *e, int64_t *poses_done, int64_t *batches, int64_t *graph_replays, int64_t *queued) {
  if (!e) return CF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(e->mu);
  if (poses_done) *poses_done = e->poses_done;
  if (batches) *batches = e->batches;
  if (graph_replays) *graph_replays = e->replays;
  if (queued) *queued = e->pending.queued_poses();
  return CF_OK;
}

const char *cf_engine_last_error(cf_engine *e) { return e ? e->last_error.c_str() : "engine is NULL"; }

void cf_engine_destroy(cf_engine *e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
  }
  e->cv.notify_all();
  if (e->worker.joinable()) e->worker.join();
  for (Slot &s : e->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  delete e;
}

}  // extern "C"
