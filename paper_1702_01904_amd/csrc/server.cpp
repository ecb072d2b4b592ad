// Serving layer: resident S-matrices under a byte budget, S-matrix builds
// and probe queries that arrive while others run, merged probe-step calls.
//
// The S-matrix of a specimen is built once (Fig. 1c) and then serves any
// number of probe positions and probe settings (the re-use of the S-matrix
// discussed in "PRISM Simulations with Varying Probe Size"). The server
// keeps the admitted S-matrices under a byte budget and host-side queues of
// builds and queries. Each flush dispatches what has arrived since the last
// one (continuous batching):
//   * builds in arrival order on the server's build stream, each admitted
//     once its bytes fit the budget; with LRU eviction on, the least
//     recently used idle S-matrices are released to make room;
//   * the queued queries of every specimen whose build has been dispatched,
//     bucketed by probe-step launch class (prism_probe_class) in arrival
//     order: one prism_probe_batch call per bucket and max_probes
//     positions, so that queries of different specimens (and optics) share
//     the window-sum and window launches, with the queries of one
//     (specimen, optics, detector) staged into one request. Each call goes
//     to the first query slot (stream) that has finished its earlier work,
//     or else to the slot with the fewest calls in flight (with a dispatch
//     limit, queries wait in the queue while every slot holds that many
//     calls, and merge with later arrivals when a slot frees up), and its
//     stream waits on the device for the build events of the S-matrices it
//     reads, so builds and queries of other specimens overlap on the GPU.
// The server is a client of the public entry points only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host_util.hpp"
#include "prism.h"

namespace {

using prism::set_error;

enum class SpecState { kBuildQueued, kResident, kReleased };

struct Specimen {
  prism_plan* plan;
  int f;
  double amax;
  const void* S;
  size_t bytes;      // prism_smatrix_bytes: what the budget counts
  size_t S_bytes;    // the caller's buffer
  hipEvent_t ready;  // recorded after the S-matrix is complete (build stream)
  SpecState state;
  long long last_use;  // dispatch sequence of the last call that read it (LRU)
  int queued;          // queued queries
  int inflight;        // dispatched calls (builds, probe steps) not yet seen finished
};

struct Query {
  long long ticket;
  int spec;
  const double* xy;
  int P;
  prism_optics optics;
  std::vector<double> edges;  // [n_det][2]
  double* out;
};

struct Build {
  long long ticket;
  int spec;
  void* ws;
  size_t ws_bytes;
};

struct Batch {
  hipEvent_t done;
  int pending;             // tickets of this batch not yet reported
  std::vector<int> specs;  // specimens it reads (or the one it builds)
  int slot;                // query slot, or -1 for the build stream
  bool finished;           // done event seen complete (specimen and slot counts released)
};

uint64_t bits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, sizeof u);
  return u;
}

}  // namespace

struct prism_server {
  size_t budget = 0, used = 0;
  int max_probes = 0, max_det = 0;
  bool lru = false;
  std::vector<hipStream_t> streams;  // query slots
  std::vector<int> slot_inflight;    // calls in flight per slot
  hipStream_t build_stream = nullptr;
  char* ws = nullptr;
  size_t region = 0;  // bytes of the workspace per query slot
  long long seq = 0;  // dispatch sequence (LRU clock)
  std::vector<Specimen> specs;
  std::vector<Query> pending;
  std::deque<Build> builds;
  long long next_ticket = 1;
  std::map<long long, int> ticket_batch;  // dispatched: ticket -> batch index
  std::vector<Batch> batches;
  std::vector<int> free_batches;  // retired batch slots
  std::vector<hipEvent_t> event_pool;
  std::vector<int> evicted;  // released by LRU eviction, not yet reported
  long long merged_calls = 0, multi_specimen_calls = 0;  // dispatched probe calls
  int dispatch_limit = 0;  // calls in flight per slot before queries wait (0: no limit)

  ~prism_server() {
    for (auto s : streams) (void)hipStreamSynchronize(s);
    if (build_stream) (void)hipStreamSynchronize(build_stream);
    for (auto& b : batches)
      if (b.done) (void)hipEventDestroy(b.done);
    for (auto e : event_pool) (void)hipEventDestroy(e);
    for (auto& s : specs)
      if (s.ready) (void)hipEventDestroy(s.ready);
    for (auto s : streams) (void)hipStreamDestroy(s);
    if (build_stream) (void)hipStreamDestroy(build_stream);
  }
  hipEvent_t event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

// Per-slot region of the server workspace: probe positions and outputs of
// one merged call, then the probe-step workspace.
struct Region {
  double* xy;
  double* out;
  void* probe_ws;
  size_t probe_ws_bytes;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t staging_bytes(int max_probes, int max_det) {
  return align256((size_t)max_probes * 2 * sizeof(double)) +
         align256((size_t)max_probes * max_det * sizeof(double));
}

Region region_of(const prism_server* s, int k) {
  char* base = s->ws + (size_t)k * s->region;
  const size_t a = align256((size_t)s->max_probes * 2 * sizeof(double));
  const size_t b = align256((size_t)s->max_probes * s->max_det * sizeof(double));
  return Region{reinterpret_cast<double*>(base), reinterpret_cast<double*>(base + a),
                base + a + b, s->region - a - b};
}

int hip_err(hipError_t e, const char* where) {
  return set_error(PRISM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// A dispatched call has finished: release what it held.
void finish(prism_server* s, Batch& bt) {
  if (bt.finished) return;
  bt.finished = true;
  for (int sp : bt.specs) s->specs[sp].inflight--;
  if (bt.slot >= 0) s->slot_inflight[bt.slot]--;
}

// Look at every dispatched call not yet seen finished.
int refresh(prism_server* s) {
  for (auto& bt : s->batches) {
    if (!bt.done || bt.finished) continue;
    const hipError_t e = hipEventQuery(bt.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return hip_err(e, "query event");
    finish(s, bt);
  }
  return PRISM_OK;
}

// Report one ticket of a batch; retire the batch when all are reported.
void recycle(prism_server* s, int b) {
  Batch& bt = s->batches[b];
  if (--bt.pending == 0) {
    finish(s, bt);
    if (bt.done) s->event_pool.push_back(bt.done);
    bt.done = nullptr;
    s->free_batches.push_back(b);
  }
}

int new_batch(prism_server* s, hipEvent_t done, int pending, std::vector<int> specs, int slot) {
  for (int sp : specs) s->specs[sp].inflight++;
  Batch bt{done, pending, std::move(specs), slot, false};
  if (slot >= 0) s->slot_inflight[slot]++;
  if (!s->free_batches.empty()) {
    const int b = s->free_batches.back();
    s->free_batches.pop_back();
    s->batches[b] = bt;
    return b;
  }
  s->batches.push_back(bt);
  return (int)s->batches.size() - 1;
}

void release(prism_server* s, int id) {
  s->specs[id].state = SpecState::kReleased;
  s->used -= s->specs[id].bytes;
}

// Make room for `need` bytes: with LRU eviction, release idle S-matrices
// (resident, no queued query, nothing in flight) least recently used first.
// Returns whether the bytes fit afterwards.
bool make_room(prism_server* s, size_t need) {
  if (s->used + need <= s->budget) return true;
  if (!s->lru || need > s->budget) return false;
  std::vector<int> idle;
  for (int i = 0; i < (int)s->specs.size(); ++i) {
    const Specimen& sp = s->specs[i];
    // idle: resident, no queued query, no call in flight, and its build
    // (an admit's build is not a tracked call) complete
    if (sp.state == SpecState::kResident && sp.queued == 0 && sp.inflight == 0 &&
        hipEventQuery(sp.ready) == hipSuccess)
      idle.push_back(i);
  }
  std::sort(idle.begin(), idle.end(),
            [&](int a, int b) { return s->specs[a].last_use < s->specs[b].last_use; });
  size_t freeable = 0;
  for (int i : idle) freeable += s->specs[i].bytes;
  if (s->used - freeable + need > s->budget) return false;  // evict nothing in vain
  for (int i : idle) {
    if (s->used + need <= s->budget) break;
    release(s, i);
    s->evicted.push_back(i);
  }
  return true;
}

// Query slot for the next call: the first one whose earlier calls have all
// finished, else the one with the fewest calls in flight; -1 when every
// slot holds dispatch_limit calls (the queries wait for the next flush).
int pick_slot(const prism_server* s) {
  int best = 0;
  for (int k = 0; k < (int)s->streams.size(); ++k) {
    if (s->slot_inflight[k] == 0) return k;
    if (s->slot_inflight[k] < s->slot_inflight[best]) best = k;
  }
  if (s->dispatch_limit > 0 && s->slot_inflight[best] >= s->dispatch_limit) return -1;
  return best;
}

int dispatch_builds(prism_server* s) {
  while (!s->builds.empty()) {
    const Build bd = s->builds.front();
    Specimen& sp = s->specs[bd.spec];
    if (!make_room(s, sp.bytes)) break;  // arrival order: later builds wait too
    s->builds.pop_front();
    hipStream_t st = s->build_stream;
    if (int r = prism_build_smatrix(sp.plan, sp.f, sp.amax, const_cast<void*>(sp.S), sp.S_bytes,
                                    bd.ws, bd.ws_bytes, st))
      return r;
    if (hipError_t e = hipEventRecord(sp.ready, st); e != hipSuccess) return hip_err(e, "record event");
    sp.state = SpecState::kResident;
    s->used += sp.bytes;
    sp.last_use = ++s->seq;
    hipEvent_t done = s->event();
    if (!done) return set_error(PRISM_EHIP, "create event");
    if (hipError_t e = hipEventRecord(done, st); e != hipSuccess) return hip_err(e, "record event");
    s->ticket_batch[bd.ticket] = new_batch(s, done, 1, {bd.spec}, -1);
  }
  return PRISM_OK;
}

// One request of a merged call: consecutive queued queries (indices into
// pending) of one (specimen, optics, detector), staged contiguously.
struct Run {
  std::vector<size_t> qs;
  int probes = 0;
};

int flush_queries(prism_server* s, std::vector<char>* sent) {
  // buckets: launch class, in arrival order; within a bucket, runs of one
  // (specimen, optics, detector)
  using Key = std::tuple<int, uint64_t, uint64_t, uint64_t, uint64_t, uint64_t, std::vector<uint64_t>>;
  std::vector<unsigned long long> cls;
  std::vector<std::vector<Key>> bucket_keys;
  std::vector<std::map<Key, std::vector<size_t>>> buckets;
  for (size_t i = 0; i < s->pending.size(); ++i) {
    const Query& q = s->pending[i];
    const Specimen& sp = s->specs[q.spec];
    if (sp.state != SpecState::kResident) continue;  // its build is still queued
    unsigned long long c;
    if (int r = prism_probe_class(sp.plan, sp.f, &c)) return r;
    size_t b = 0;
    while (b < cls.size() && cls[b] != c) ++b;
    if (b == cls.size()) {
      cls.push_back(c);
      bucket_keys.emplace_back();
      buckets.emplace_back();
    }
    std::vector<uint64_t> eb;
    for (double e : q.edges) eb.push_back(bits(e));
    Key k{q.spec, bits(q.optics.alpha_mrad), bits(q.optics.C1_A), bits(q.optics.C3_A),
          bits(q.optics.tilt_x_mrad), bits(q.optics.tilt_y_mrad), eb};
    auto it = buckets[b].find(k);
    if (it == buckets[b].end()) {
      bucket_keys[b].push_back(k);
      buckets[b][k] = {i};
    } else {
      it->second.push_back(i);
    }
  }
  for (size_t b = 0; b < cls.size(); ++b) {
    // the bucket's runs, cut so that a call holds at most max_probes positions
    std::vector<Run> runs;
    for (const Key& k : bucket_keys[b]) {
      Run cur;
      for (size_t i : buckets[b][k]) {
        const int P = s->pending[i].P;
        if (cur.probes + P > s->max_probes && !cur.qs.empty()) {
          runs.push_back(std::move(cur));
          cur = Run{};
        }
        cur.qs.push_back(i);
        cur.probes += P;
      }
      if (!cur.qs.empty()) runs.push_back(std::move(cur));
    }
    size_t r0 = 0;
    while (r0 < runs.size()) {
      // one call: consecutive runs up to max_probes positions
      size_t r1 = r0;
      int total = 0;
      while (r1 < runs.size() && total + runs[r1].probes <= s->max_probes) total += runs[r1++].probes;
      const int k_st = pick_slot(s);
      if (k_st < 0) return PRISM_OK;  // every slot busy: the rest stays queued
      hipStream_t st = s->streams[k_st];
      const Region rg = region_of(s, k_st);
      std::vector<int> specs;
      for (size_t r = r0; r < r1; ++r) {
        const int sid = s->pending[runs[r].qs[0]].spec;
        if (std::find(specs.begin(), specs.end(), sid) == specs.end()) specs.push_back(sid);
      }
      for (int sid : specs)
        if (hipError_t e = hipStreamWaitEvent(st, s->specs[sid].ready, 0); e != hipSuccess)
          return hip_err(e, "wait S-matrix");
      // stage positions, then one request per run
      std::vector<prism_detector> dets(r1 - r0);
      std::vector<prism_probe_request> req(r1 - r0);
      int off = 0;  // staged positions so far (output rows follow them at max_det each)
      std::vector<int> offs;
      for (size_t r = r0; r < r1; ++r) {
        offs.push_back(off);
        const Query& q0 = s->pending[runs[r].qs[0]];
        const Specimen& sp = s->specs[q0.spec];
        int o = off;
        for (size_t i : runs[r].qs) {
          const Query& q = s->pending[i];
          if (q.P > 0)
            if (hipError_t e = hipMemcpyAsync(rg.xy + 2 * (size_t)o, q.xy,
                                              2 * (size_t)q.P * sizeof(double),
                                              hipMemcpyDeviceToDevice, st);
                e != hipSuccess)
              return hip_err(e, "stage probe positions");
          o += q.P;
        }
        const int n_det = (int)(q0.edges.size() / 2);
        dets[r - r0] = prism_detector{n_det, q0.edges.data()};
        req[r - r0] = prism_probe_request{sp.plan, sp.f, sp.amax, sp.S, sp.S_bytes,
                                          rg.xy + 2 * (size_t)off, runs[r].probes, &q0.optics,
                                          &dets[r - r0], rg.out + (size_t)off * s->max_det,
                                          nullptr, 0, 1.0};
        off += runs[r].probes;
      }
      if (total > 0)
        if (int e = prism_probe_batch(req.data(), (int)req.size(), rg.probe_ws, rg.probe_ws_bytes,
                                      st))
          return e;
      for (size_t r = r0; r < r1; ++r) {
        const int n_det = dets[r - r0].n_det;
        int o = 0;
        for (size_t i : runs[r].qs) {
          const Query& q = s->pending[i];
          if (q.P > 0)
            if (hipError_t e = hipMemcpyAsync(
                    q.out, rg.out + (size_t)offs[r - r0] * s->max_det + (size_t)o * n_det,
                    (size_t)q.P * n_det * sizeof(double), hipMemcpyDeviceToDevice, st);
                e != hipSuccess)
              return hip_err(e, "return outputs");
          o += q.P;
        }
      }
      hipEvent_t done = s->event();
      if (!done) return set_error(PRISM_EHIP, "create event");
      if (hipError_t e = hipEventRecord(done, st); e != hipSuccess) return hip_err(e, "record event");
      int n_q = 0;
      for (size_t r = r0; r < r1; ++r) n_q += (int)runs[r].qs.size();
      const int bi = new_batch(s, done, n_q, specs, k_st);
      ++s->seq;
      for (int sid : specs) s->specs[sid].last_use = s->seq;
      for (size_t r = r0; r < r1; ++r)
        for (size_t i : runs[r].qs) {
          s->ticket_batch[s->pending[i].ticket] = bi;
          (*sent)[i] = 1;
          s->specs[s->pending[i].spec].queued--;
        }
      s->merged_calls++;
      if (specs.size() > 1) s->multi_specimen_calls++;
      r0 = r1;
    }
  }
  return PRISM_OK;
}

bool live_id(const prism_server* s, int id) {
  return id >= 0 && id < (int)s->specs.size() && s->specs[id].state != SpecState::kReleased;
}

// Register a specimen (its ready event included); *id names it.
int add_specimen(prism_server* s, prism_plan* plan, int f, double amax, void* S, size_t bytes,
                 size_t S_bytes, SpecState state, int* id) {
  hipEvent_t ready = nullptr;
  if (hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming); e != hipSuccess)
    return hip_err(e, "create event");
  s->specs.push_back(Specimen{plan, f, amax, S, bytes, S_bytes, ready, state, 0, 0, 0});
  *id = (int)s->specs.size() - 1;
  return PRISM_OK;
}

}  // namespace

extern "C" {

int prism_server_workspace_bytes(int n_streams, int max_probes, int max_det,
                                 size_t probe_ws_bytes, size_t* bytes) {
  if (!bytes) return set_error(PRISM_EINVAL, "null argument");
  if (n_streams < 1 || n_streams > 16) return set_error(PRISM_EINVAL, "n_streams must be 1..16");
  if (max_probes < 1) return set_error(PRISM_EINVAL, "max_probes must be >= 1");
  if (max_det < 1 || max_det > PRISM_MAX_DET) return set_error(PRISM_EINVAL, "max_det out of range");
  *bytes = (size_t)n_streams * align256(staging_bytes(max_probes, max_det) + probe_ws_bytes) + 256;
  return PRISM_OK;
}

int prism_server_create(prism_server** out, size_t smatrix_budget_bytes, int n_streams,
                        int max_probes, int max_det, void* ws, size_t ws_bytes) {
  if (!out) return set_error(PRISM_EINVAL, "null argument");
  *out = nullptr;
  size_t need;
  if (int r = prism_server_workspace_bytes(n_streams, max_probes, max_det, 0, &need)) return r;
  if (!ws) return set_error(PRISM_EINVAL, "null workspace");
  if (ws_bytes < need) return set_error(PRISM_ENOSPACE, "server workspace below its staging size");
  auto* s = new prism_server();
  s->budget = smatrix_budget_bytes;
  s->max_probes = max_probes;
  s->max_det = max_det;
  const uintptr_t u = reinterpret_cast<uintptr_t>(ws);
  const uintptr_t a = (u + 255) & ~uintptr_t(255);
  s->ws = reinterpret_cast<char*>(a);
  s->region = ((ws_bytes - (a - u)) / n_streams) & ~size_t(255);
  for (int k = 0; k <= n_streams; ++k) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return hip_err(e, "create server stream");
    }
    if (k < n_streams) {
      s->streams.push_back(st);
      s->slot_inflight.push_back(0);
    } else {
      s->build_stream = st;
    }
  }
  *out = s;
  return PRISM_OK;
}

void prism_server_destroy(prism_server* s) { delete s; }

int prism_server_set_lru_eviction(prism_server* s, int enable) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  s->lru = enable != 0;
  return PRISM_OK;
}

int prism_server_admit(prism_server* s, prism_plan* plan, int f, double alpha_max_mrad,
                       void* smatrix_dev, size_t smatrix_bytes, void* build_ws,
                       size_t build_ws_bytes, int* id) {
  if (!s || !plan || !smatrix_dev || !id) return set_error(PRISM_EINVAL, "null argument");
  size_t bytes;
  if (int r = prism_smatrix_bytes(plan, f, alpha_max_mrad, &bytes)) return r;
  if (smatrix_bytes < bytes)
    return set_error(PRISM_EINVAL, "S-matrix buffer smaller than prism_smatrix_bytes");
  if (int r = refresh(s)) return r;
  if (!make_room(s, bytes))
    return set_error(PRISM_ENOSPACE, "S-matrix does not fit in the server's budget");
  // builds run on the server's build stream, in the order they are given
  hipStream_t st = s->build_stream;
  if (build_ws) {
    if (int r = prism_build_smatrix(plan, f, alpha_max_mrad, smatrix_dev, smatrix_bytes,
                                    build_ws, build_ws_bytes, st))
      return r;
  }
  int sid;
  if (int r = add_specimen(s, plan, f, alpha_max_mrad, smatrix_dev, bytes, smatrix_bytes,
                           SpecState::kResident, &sid))
    return r;
  if (hipError_t e = hipEventRecord(s->specs[sid].ready, st); e != hipSuccess)
    return hip_err(e, "record event");
  s->used += bytes;
  s->specs[sid].last_use = ++s->seq;
  *id = sid;
  return PRISM_OK;
}

int prism_server_submit_build(prism_server* s, prism_plan* plan, int f, double alpha_max_mrad,
                              void* smatrix_dev, size_t smatrix_bytes, void* build_ws,
                              size_t build_ws_bytes, int* id, long long* ticket) {
  if (!s || !plan || !smatrix_dev || !build_ws || !id || !ticket)
    return set_error(PRISM_EINVAL, "null argument");
  size_t bytes, pref, minimum;
  if (int r = prism_smatrix_bytes(plan, f, alpha_max_mrad, &bytes)) return r;
  if (smatrix_bytes < bytes)
    return set_error(PRISM_EINVAL, "S-matrix buffer smaller than prism_smatrix_bytes");
  if (bytes > s->budget)
    return set_error(PRISM_ENOSPACE, "S-matrix larger than the server's whole budget");
  if (int r = prism_build_workspace_bytes(plan, f, alpha_max_mrad, &pref, &minimum)) return r;
  if (build_ws_bytes < minimum)
    return set_error(PRISM_ENOSPACE, "build workspace smaller than the build minimum");
  int sid;
  if (int r = add_specimen(s, plan, f, alpha_max_mrad, smatrix_dev, bytes, smatrix_bytes,
                           SpecState::kBuildQueued, &sid))
    return r;
  const long long t = s->next_ticket++;
  s->builds.push_back(Build{t, sid, build_ws, build_ws_bytes});
  *id = sid;
  *ticket = t;
  return PRISM_OK;
}

int prism_server_evict(prism_server* s, int id) {
  if (!s || !live_id(s, id)) return set_error(PRISM_EINVAL, "no such specimen");
  if (s->specs[id].state == SpecState::kBuildQueued)
    return set_error(PRISM_EINVAL, "specimen's build is still queued");
  if (s->specs[id].queued > 0) return set_error(PRISM_EINVAL, "specimen has queued queries");
  // calls already dispatched must finish before the caller reuses the memory
  for (auto st : s->streams)
    if (hipError_t e = hipStreamSynchronize(st); e != hipSuccess) return hip_err(e, "drain");
  if (hipError_t e = hipStreamSynchronize(s->build_stream); e != hipSuccess) return hip_err(e, "drain");
  if (int r = refresh(s)) return r;
  release(s, id);
  return PRISM_OK;
}

int prism_server_set_dispatch_limit(prism_server* s, int calls_per_slot) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  if (calls_per_slot < 0) return set_error(PRISM_EINVAL, "calls_per_slot must be >= 0");
  s->dispatch_limit = calls_per_slot;
  return PRISM_OK;
}

int prism_server_evictions(prism_server* s, int* ids, int capacity, int* count) {
  if (!s || !count || (capacity > 0 && !ids)) return set_error(PRISM_EINVAL, "null argument");
  const int n = std::min(capacity, (int)s->evicted.size());
  for (int i = 0; i < n; ++i) ids[i] = s->evicted[i];
  s->evicted.erase(s->evicted.begin(), s->evicted.begin() + n);
  *count = n;
  return PRISM_OK;
}

int prism_server_submit(prism_server* s, int id, const double* probe_xy_dev, int n_probes,
                        const prism_optics* optics, const prism_detector* detector,
                        double* out_dev, long long* ticket) {
  if (!s || !optics || !detector || !ticket) return set_error(PRISM_EINVAL, "null argument");
  if (!live_id(s, id)) return set_error(PRISM_EINVAL, "no such specimen");
  if (n_probes < 0 || n_probes > s->max_probes)
    return set_error(PRISM_EINVAL, "probe count must be 0..max_probes");
  if (detector->n_det < 1 || detector->n_det > s->max_det || !detector->edges_mrad)
    return set_error(PRISM_EINVAL, "detector bins must be 1..max_det");
  // the probe step's bin checks, here so that a bad query never reaches a flush
  for (int j = 0; j < detector->n_det; ++j) {
    const double lo = detector->edges_mrad[2 * j], hi = detector->edges_mrad[2 * j + 1];
    if (!std::isfinite(lo) || !std::isfinite(hi) || lo < 0.0 || hi < lo)
      return set_error(PRISM_EINVAL, "detector edges must satisfy 0 <= inner <= outer");
  }
  if (n_probes > 0 && (!probe_xy_dev || !out_dev)) return set_error(PRISM_EINVAL, "null device buffer");
  Specimen& sp = s->specs[id];
  if (optics->alpha_mrad + std::hypot(optics->tilt_x_mrad, optics->tilt_y_mrad) > sp.amax)
    return set_error(PRISM_EINVAL, "probe semi-angle plus tilt exceeds the beam set's alpha_max");
  // the probe step's own checks, and its workspace minimum against a region
  size_t pref, minimum;
  if (int r = prism_probe_workspace_bytes(sp.plan, sp.f, sp.amax, optics, &pref, &minimum)) return r;
  if (minimum > region_of(s, 0).probe_ws_bytes)
    return set_error(PRISM_ENOSPACE, "server workspace region below the probe-step minimum");
  Query q{s->next_ticket++, id, probe_xy_dev, n_probes, *optics,
          std::vector<double>(detector->edges_mrad, detector->edges_mrad + 2 * detector->n_det),
          out_dev};
  *ticket = q.ticket;
  sp.queued++;
  s->pending.push_back(std::move(q));
  return PRISM_OK;
}

int prism_server_flush(prism_server* s) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  if (int r = refresh(s)) return r;
  int r = dispatch_builds(s);
  std::vector<char> sent(s->pending.size(), 0);
  if (r == PRISM_OK) r = flush_queries(s, &sent);
  // dispatched queries leave the queue even when a later group failed
  std::vector<Query> keep;
  for (size_t i = 0; i < s->pending.size(); ++i)
    if (!sent[i]) keep.push_back(std::move(s->pending[i]));
  s->pending.swap(keep);
  return r;
}

int prism_server_poll(prism_server* s, long long* done, int capacity, int* count) {
  if (!s || !count || (capacity > 0 && !done)) return set_error(PRISM_EINVAL, "null argument");
  *count = 0;
  if (int r = refresh(s)) return r;
  for (auto it = s->ticket_batch.begin(); it != s->ticket_batch.end() && *count < capacity;) {
    if (!s->batches[it->second].finished) {
      ++it;
      continue;
    }
    done[(*count)++] = it->first;
    const int b = it->second;
    it = s->ticket_batch.erase(it);
    recycle(s, b);
  }
  return PRISM_OK;
}

int prism_server_wait(prism_server* s, long long ticket) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  for (const Query& q : s->pending)
    if (q.ticket == ticket) return set_error(PRISM_EINVAL, "query not flushed yet");
  for (const Build& b : s->builds)
    if (b.ticket == ticket) return set_error(PRISM_EINVAL, "build not dispatched yet");
  auto it = s->ticket_batch.find(ticket);
  if (it == s->ticket_batch.end()) return set_error(PRISM_EINVAL, "unknown or already reported ticket");
  Batch& bt = s->batches[it->second];
  if (bt.done && !bt.finished)
    if (hipError_t e = hipEventSynchronize(bt.done); e != hipSuccess) return hip_err(e, "wait");
  finish(s, bt);
  const int b = it->second;
  s->ticket_batch.erase(it);
  recycle(s, b);
  return PRISM_OK;
}

int prism_server_stats(const prism_server* s, size_t* smatrix_bytes_used, int* queued,
                       int* in_flight) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  if (smatrix_bytes_used) *smatrix_bytes_used = s->used;
  if (queued) *queued = (int)(s->pending.size() + s->builds.size());
  if (in_flight) *in_flight = (int)s->ticket_batch.size();
  return PRISM_OK;
}

int prism_server_call_stats(const prism_server* s, long long* probe_calls,
                            long long* multi_specimen_calls) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  if (probe_calls) *probe_calls = s->merged_calls;
  if (multi_specimen_calls) *multi_specimen_calls = s->multi_specimen_calls;
  return PRISM_OK;
}

}  // extern "C"
