// Serving layer: resident S-matrices under a byte budget and a queue of
// probe queries that are merged into shared probe-step calls.
//
// The S-matrix of a specimen is built once (Fig. 1c) and then serves any
// number of probe positions and probe settings (the re-use of the S-matrix
// discussed in "PRISM Simulations with Varying Probe Size"). The server
// keeps a set of admitted S-matrices whose bytes stay under a budget and a
// host-side queue of queries. prism_server_flush merges every pending query
// of one (specimen, optics, detector) into as few probe-step calls as the
// staging space allows (continuous batching: what arrived since the last
// flush rides in the same launches) and spreads the merged calls over the
// server's streams. The server is a client of the public entry points only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host_util.hpp"
#include "prism.h"

namespace {

using prism::set_error;

struct Specimen {
  prism_plan* plan;
  int f;
  double amax;
  const void* S;
  size_t bytes;     // prism_smatrix_bytes: what the budget counts
  size_t S_bytes;   // the caller's buffer
  hipEvent_t ready;
  bool live;
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

struct Batch {
  hipEvent_t done;
  int pending;  // tickets of this batch not yet reported
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
  std::vector<hipStream_t> streams;
  char* ws = nullptr;
  size_t region = 0;  // bytes of the workspace per stream
  int next_stream = 0;
  std::vector<Specimen> specs;
  std::vector<Query> pending;
  long long next_ticket = 1;
  std::map<long long, int> ticket_batch;  // in flight: ticket -> batch index
  std::vector<Batch> batches;
  std::vector<int> free_batches;  // retired batch slots
  std::vector<hipEvent_t> event_pool;

  ~prism_server() {
    for (auto s : streams) (void)hipStreamSynchronize(s);
    for (auto& b : batches)
      if (b.done) (void)hipEventDestroy(b.done);
    for (auto e : event_pool) (void)hipEventDestroy(e);
    for (auto& s : specs)
      if (s.ready) (void)hipEventDestroy(s.ready);
    for (auto s : streams) (void)hipStreamDestroy(s);
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

// Per-stream region of the server workspace: probe positions and outputs of
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

// Retire finished batches: their tickets are reported done by poll/wait.
void recycle(prism_server* s, int b) {
  if (--s->batches[b].pending == 0) {
    if (s->batches[b].done) s->event_pool.push_back(s->batches[b].done);
    s->batches[b].done = nullptr;
    s->free_batches.push_back(b);
  }
}

int new_batch(prism_server* s, hipEvent_t done, int pending) {
  if (!s->free_batches.empty()) {
    const int b = s->free_batches.back();
    s->free_batches.pop_back();
    s->batches[b] = Batch{done, pending};
    return b;
  }
  s->batches.push_back(Batch{done, pending});
  return (int)s->batches.size() - 1;
}

int flush_groups(prism_server* s, std::vector<char>* sent) {
  // merge key: specimen, optics, detector; queries keep their arrival order
  using Key = std::tuple<int, uint64_t, uint64_t, uint64_t, uint64_t, uint64_t, std::vector<uint64_t>>;
  std::map<Key, std::vector<size_t>> groups;
  std::vector<Key> order;
  for (size_t i = 0; i < s->pending.size(); ++i) {
    const Query& q = s->pending[i];
    std::vector<uint64_t> eb;
    for (double e : q.edges) eb.push_back(bits(e));
    Key k{q.spec, bits(q.optics.alpha_mrad), bits(q.optics.C1_A), bits(q.optics.C3_A),
          bits(q.optics.tilt_x_mrad), bits(q.optics.tilt_y_mrad), eb};
    auto it = groups.find(k);
    if (it == groups.end()) {
      order.push_back(k);
      groups[k] = {i};
    } else {
      it->second.push_back(i);
    }
  }
  for (const Key& k : order) {
    const std::vector<size_t>& qs = groups[k];
    size_t a = 0;
    while (a < qs.size()) {
      // one merged call: consecutive queries up to max_probes positions
      size_t b = a;
      int total = 0;
      while (b < qs.size() && total + s->pending[qs[b]].P <= s->max_probes) total += s->pending[qs[b++]].P;
      const Query& q0 = s->pending[qs[a]];
      const Specimen& sp = s->specs[q0.spec];
      const int n_det = (int)(q0.edges.size() / 2);
      const int k_st = s->next_stream;
      s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
      hipStream_t st = s->streams[k_st];
      const Region rg = region_of(s, k_st);
      if (hipError_t e = hipStreamWaitEvent(st, sp.ready, 0); e != hipSuccess) return hip_err(e, "wait S-matrix");
      int off = 0;
      for (size_t i = a; i < b; ++i) {
        const Query& q = s->pending[qs[i]];
        if (q.P > 0)
          if (hipError_t e = hipMemcpyAsync(rg.xy + 2 * (size_t)off, q.xy, 2 * (size_t)q.P * sizeof(double),
                                            hipMemcpyDeviceToDevice, st);
              e != hipSuccess)
            return hip_err(e, "stage probe positions");
        off += q.P;
      }
      prism_detector det{n_det, q0.edges.data()};
      if (total > 0)
        if (int r = prism_probe_outputs(sp.plan, sp.f, sp.amax, sp.S, sp.S_bytes, rg.xy, total,
                                        &q0.optics, &det, rg.out, rg.probe_ws, rg.probe_ws_bytes,
                                        st))
          return r;
      off = 0;
      for (size_t i = a; i < b; ++i) {
        const Query& q = s->pending[qs[i]];
        if (q.P > 0)
          if (hipError_t e = hipMemcpyAsync(q.out, rg.out + (size_t)off * n_det,
                                            (size_t)q.P * n_det * sizeof(double),
                                            hipMemcpyDeviceToDevice, st);
              e != hipSuccess)
            return hip_err(e, "return outputs");
        off += q.P;
      }
      hipEvent_t done = s->event();
      if (!done) return set_error(PRISM_EHIP, "create event");
      if (hipError_t e = hipEventRecord(done, st); e != hipSuccess) return hip_err(e, "record event");
      const int bi = new_batch(s, done, (int)(b - a));
      for (size_t i = a; i < b; ++i) {
        s->ticket_batch[s->pending[qs[i]].ticket] = bi;
        (*sent)[qs[i]] = 1;
      }
      a = b;
    }
  }
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
  for (int k = 0; k < n_streams; ++k) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return hip_err(e, "create server stream");
    }
    s->streams.push_back(st);
  }
  *out = s;
  return PRISM_OK;
}

void prism_server_destroy(prism_server* s) { delete s; }

int prism_server_admit(prism_server* s, prism_plan* plan, int f, double alpha_max_mrad,
                       void* smatrix_dev, size_t smatrix_bytes, void* build_ws,
                       size_t build_ws_bytes, int* id) {
  if (!s || !plan || !smatrix_dev || !id) return set_error(PRISM_EINVAL, "null argument");
  size_t bytes;
  if (int r = prism_smatrix_bytes(plan, f, alpha_max_mrad, &bytes)) return r;
  if (smatrix_bytes < bytes)
    return set_error(PRISM_EINVAL, "S-matrix buffer smaller than prism_smatrix_bytes");
  if (s->used + bytes > s->budget)
    return set_error(PRISM_ENOSPACE, "S-matrix does not fit in the server's budget");
  // every build runs on the server's first stream, so builds are ordered
  // among themselves (two builds may share one build workspace)
  hipStream_t st = s->streams[0];
  if (build_ws) {
    if (int r = prism_build_smatrix(plan, f, alpha_max_mrad, smatrix_dev, smatrix_bytes,
                                    build_ws, build_ws_bytes, st))
      return r;
  }
  hipEvent_t ready = s->event();
  if (!ready) return set_error(PRISM_EHIP, "create event");
  if (hipError_t e = hipEventRecord(ready, st); e != hipSuccess) return hip_err(e, "record event");
  s->specs.push_back(Specimen{plan, f, alpha_max_mrad, smatrix_dev, bytes, smatrix_bytes, ready,
                              true});
  s->used += bytes;
  *id = (int)s->specs.size() - 1;
  return PRISM_OK;
}

int prism_server_evict(prism_server* s, int id) {
  if (!s || id < 0 || id >= (int)s->specs.size() || !s->specs[id].live)
    return set_error(PRISM_EINVAL, "no such specimen");
  for (const Query& q : s->pending)
    if (q.spec == id) return set_error(PRISM_EINVAL, "specimen has queued queries");
  // queries already dispatched must finish before the caller reuses the memory
  for (auto st : s->streams)
    if (hipError_t e = hipStreamSynchronize(st); e != hipSuccess) return hip_err(e, "drain");
  s->specs[id].live = false;
  s->used -= s->specs[id].bytes;
  return PRISM_OK;
}

int prism_server_submit(prism_server* s, int id, const double* probe_xy_dev, int n_probes,
                        const prism_optics* optics, const prism_detector* detector,
                        double* out_dev, long long* ticket) {
  if (!s || !optics || !detector || !ticket) return set_error(PRISM_EINVAL, "null argument");
  if (id < 0 || id >= (int)s->specs.size() || !s->specs[id].live)
    return set_error(PRISM_EINVAL, "no such specimen");
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
  const Specimen& sp = s->specs[id];
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
  s->pending.push_back(std::move(q));
  return PRISM_OK;
}

int prism_server_flush(prism_server* s) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  std::vector<char> sent(s->pending.size(), 0);
  const int r = flush_groups(s, &sent);
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
  for (auto it = s->ticket_batch.begin(); it != s->ticket_batch.end() && *count < capacity;) {
    Batch& bt = s->batches[it->second];
    const hipError_t e = bt.done ? hipEventQuery(bt.done) : hipSuccess;
    if (e == hipErrorNotReady) {
      ++it;
      continue;
    }
    if (e != hipSuccess) return hip_err(e, "query event");
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
  auto it = s->ticket_batch.find(ticket);
  if (it == s->ticket_batch.end()) return set_error(PRISM_EINVAL, "unknown or already reported ticket");
  Batch& bt = s->batches[it->second];
  if (bt.done)
    if (hipError_t e = hipEventSynchronize(bt.done); e != hipSuccess) return hip_err(e, "wait");
  const int b = it->second;
  s->ticket_batch.erase(it);
  recycle(s, b);
  return PRISM_OK;
}

int prism_server_stats(const prism_server* s, size_t* smatrix_bytes_used, int* queued,
                       int* in_flight) {
  if (!s) return set_error(PRISM_EINVAL, "null server");
  if (smatrix_bytes_used) *smatrix_bytes_used = s->used;
  if (queued) *queued = (int)s->pending.size();
  if (in_flight) *in_flight = (int)s->ticket_batch.size();
  return PRISM_OK;
}

}  // extern "C"
