// Host side of libprism: plans, argument checks, workspace layout, chunked
// launch sequences and the C ABI declared in include/prism.h.
//
// The plan holds only host state (grid, optics-independent constants,
// cached beam sets). Every device buffer comes from the caller; each call
// carves its workspace with a bump allocator that runs the same code for
// the size queries and for the real calls.
#include "prism.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "host_util.hpp"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

int prism::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

int hip_fail(hipError_t e, const char* where) {
  return fail(PRISM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr double kHcKeVA = 12.398419843320026;  // h c (keV A), CODATA 2018
constexpr double kMec2KeV = 510.99895000;       // electron rest energy (keV)
constexpr long long kK2Cap = 1LL << 30;

uint64_t dbits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, sizeof u);
  return u;
}

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

// Bump allocator over a caller workspace (base == nullptr: size query).
struct Carve {
  char* base;
  size_t used = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct ProfRecord {
  const char* name;
  hipEvent_t start, stop;
};

struct prism_plan {
  // per-kernel timing (prism_profile_enable / prism_profile_report)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRecord> prof;
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (!ev_pool.empty()) {
      e = ev_pool.back();
      ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // second stream of the S-matrix build (created on first use, default
  // priority) and the events that fork it from and join it to the caller's
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  ~prism_plan() {
    if (aux) (void)hipStreamDestroy(aux);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    for (auto& r : prof) {
      if (r.start) (void)hipEventDestroy(r.start);
      if (r.stop) (void)hipEventDestroy(r.stop);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }

  int n = 0;
  int prec = PRISM_PREC_FP32;  // operand precision of the probe-step window sum
  // launch shapes (prism_set_tuning): none of them changes a result
  prism::LaunchTuning tune;
  size_t wave_chunk_bytes = size_t(256) << 20;  // wave state per slice-pass launch
  int probe_group = 0;                           // probes per window-sum group (0: by W)
  double cell = 0, energy = 0, lam = 0, dq = 0;
  double height = 0;           // total slice thickness (A)
  int H = 0;
  std::vector<double> thick;
  const float* phase = nullptr;
  std::map<std::pair<int, uint64_t>, std::vector<int32_t>> beams;  // (f, alpha_max) -> [B][2]
  std::map<std::tuple<int, uint64_t, uint64_t, uint64_t, uint64_t>, std::vector<prism::ActiveBeam>>
      active;
  struct PixLists {
    std::vector<uint16_t> pix;
    prism::BinLists lists;
  };
  std::map<std::string, PixLists> pixlists;  // window detector bin lists
  // multislice aperture rows per (alpha, tilt) and their pixel count: kept
  // here because the asynchronous copy to the device reads them after the
  // call returns. An entry is filled once, when inserted, and never
  // rewritten, so a copy still queued by an earlier call reads what it was
  // given.
  struct AperRows {
    std::vector<int32_t> rows;
    long long count = 0;
  };
  std::map<std::tuple<uint64_t, uint64_t, uint64_t>, AperRows> aper_rows;
  // per-wave tables of batched builds led by this plan (same reason: the
  // asynchronous copies read them later); set nodes keep their addresses
  std::set<std::vector<uint64_t>> batch_tables;

  // scattering angle (rad) of integer full-grid |k|^2
  double theta(long long k2) const { return (lam * dq) * std::sqrt((double)k2); }
  // tilt as a full-grid frequency offset (theta_t / (lambda dq))
  double tilt_k(double tilt_mrad) const { return tilt_mrad * 1e-3 / (lam * dq); }
  // probe aperture test of full-grid frequency (kx, ky) for a tilted probe:
  // (lambda dq) |k - k_t| <= alpha, the same FP64 expression as the oracle's
  bool in_aperture(long long kx, long long ky, const prism_optics* o) const {
    const double dx = (double)kx - tilt_k(o->tilt_x_mrad), dy = (double)ky - tilt_k(o->tilt_y_mrad);
    return (lam * dq) * std::sqrt(dx * dx + dy * dy) <= o->alpha_mrad * 1e-3;
  }

  // smallest k2 >= 0 with theta(k2) >= ang
  long long first_ge(double ang) const {
    if (!(ang > 0.0)) return 0;
    const double x = ang / (lam * dq);
    if (x * x > (double)kK2Cap) return kK2Cap;
    long long k = std::max(0LL, (long long)std::floor(x * x) - 4);
    while (k > 0 && theta(k - 1) >= ang) --k;
    while (theta(k) < ang) ++k;
    return k;
  }
  // largest k2 with theta(k2) <= ang (-1 if none)
  long long last_le(double ang) const {
    if (ang < 0.0) return -1;
    const double x = ang / (lam * dq);
    if (x * x > (double)kK2Cap) return kK2Cap;
    long long k = (long long)std::floor(x * x) + 4;
    while (theta(k) > ang) --k;
    while (theta(k + 1) <= ang) ++k;
    return k;
  }
};

namespace {

int check_f(const prism_plan* p, int f) {
  if (f < 1) return fail(PRISM_EINVAL, "interpolation factor f must be >= 1");
  if (p->n % (2 * f) != 0) return fail(PRISM_EINVAL, "n must be divisible by 2 f");
  return PRISM_OK;
}

const std::vector<int32_t>* get_beams(prism_plan* p, int f, double amax_mrad) {
  const auto key = std::make_pair(f, dbits(amax_mrad));
  auto it = p->beams.find(key);
  if (it != p->beams.end()) return &it->second;
  const double amax = amax_mrad * 1e-3;
  const int lim = p->n / (4 * f) + 1;
  std::vector<int32_t> mn;
  for (int m = -lim; m <= lim; ++m)
    for (int k = -lim; k <= lim; ++k) {
      const long long k2 = (long long)(m * f) * (m * f) + (long long)(k * f) * (k * f);
      if (16 * k2 >= (long long)p->n * p->n) continue;
      if (p->theta(k2) <= amax) {
        mn.push_back(m);
        mn.push_back(k);
      }
    }
  return &(p->beams[key] = std::move(mn));
}

int beams_checked(const prism_plan* cp, int f, double amax_mrad, const std::vector<int32_t>** out) {
  prism_plan* p = const_cast<prism_plan*>(cp);
  if (!p) return fail(PRISM_EINVAL, "null plan");
  if (int r = check_f(p, f)) return r;
  if (!(amax_mrad > 0.0) || !std::isfinite(amax_mrad))
    return fail(PRISM_EINVAL, "alpha_max_mrad must be positive and finite");
  *out = get_beams(p, f, amax_mrad);
  if ((*out)->empty()) return fail(PRISM_EINVAL, "empty beam set");
  return PRISM_OK;
}

// Bytes of the compact S-matrix of a beam set: c64 [B][n/2][n/2].
size_t smatrix_need(const prism_plan* p, const std::vector<int32_t>& mn) {
  return (mn.size() / 2) * (size_t)(p->n / 2) * (p->n / 2) * sizeof(float2);
}

// Per-row kx interval of the (tilted) aperture over full-grid rows
// ky = -n/2 .. n/2-1, and its pixel count. A row of a disc is one interval.
long long aperture_rows(const prism_plan* p, const prism_optics* o, std::vector<int32_t>* rows) {
  const int n = p->n;
  if (rows) rows->assign(2 * (size_t)n, 0);
  const double ktx = p->tilt_k(o->tilt_x_mrad), kty = p->tilt_k(o->tilt_y_mrad);
  const double ka = o->alpha_mrad * 1e-3 / (p->lam * p->dq);
  long long cnt = 0;
  for (int ky = -n / 2; ky < n / 2; ++ky) {
    int lo = 1, hi = 0;  // empty
    if (std::fabs(ky - kty) <= ka + 1.0) {
      const long long x0 = (long long)std::floor(ktx - ka) - 1, x1 = (long long)std::ceil(ktx + ka) + 1;
      for (long long kx = std::max<long long>(x0, -n / 2); kx <= std::min<long long>(x1, n / 2 - 1); ++kx)
        if (p->in_aperture(kx, ky, o)) {
          if (lo > hi) lo = hi = (int)kx;
          else hi = (int)kx;
          ++cnt;
        }
    }
    if (rows) {
      (*rows)[2 * (size_t)(ky + n / 2)] = lo;
      (*rows)[2 * (size_t)(ky + n / 2) + 1] = hi;
    }
  }
  return cnt;
}

int check_optics(const prism_plan* p, const prism_optics* o) {
  if (!o) return fail(PRISM_EINVAL, "null optics");
  if (!(o->alpha_mrad > 0.0) || !std::isfinite(o->alpha_mrad) || !std::isfinite(o->C1_A) ||
      !std::isfinite(o->C3_A) || !std::isfinite(o->tilt_x_mrad) || !std::isfinite(o->tilt_y_mrad))
    return fail(PRISM_EINVAL, "optics: alpha must be positive; C1, C3 and tilt finite");
  // every aperture pixel strictly inside the half-band limit |k| < n/4 (the
  // compact wave state stores nothing beyond it)
  const double ktx = p->tilt_k(o->tilt_x_mrad), kty = p->tilt_k(o->tilt_y_mrad);
  const double ka = o->alpha_mrad * 1e-3 / (p->lam * p->dq);
  if (std::hypot(ktx, kty) + ka >= p->n / 4.0 + 2.0)
    return fail(PRISM_EINVAL, "probe aperture must lie inside the half-band anti-aliasing limit");
  const long long n2 = (long long)p->n * p->n;
  const long long y0 = (long long)std::floor(kty - ka) - 1, y1 = (long long)std::ceil(kty + ka) + 1;
  const long long x0 = (long long)std::floor(ktx - ka) - 1, x1 = (long long)std::ceil(ktx + ka) + 1;
  for (long long ky = y0; ky <= y1; ++ky)
    for (long long kx = x0; kx <= x1; ++kx)
      if (p->in_aperture(kx, ky, o) && 16 * (kx * kx + ky * ky) >= n2)
        return fail(PRISM_EINVAL, "probe aperture must lie inside the half-band anti-aliasing limit");
  return PRISM_OK;
}

int make_bins(const prism_plan* p, const prism_detector* d, prism::DetBins* b) {
  if (!d || !d->edges_mrad) return fail(PRISM_EINVAL, "null detector");
  if (d->n_det < 1 || d->n_det > PRISM_MAX_DET)
    return fail(PRISM_EINVAL, "n_det must be in [1, PRISM_MAX_DET]");
  std::memset(b, 0, sizeof *b);
  b->n = d->n_det;
  for (int j = 0; j < d->n_det; ++j) {
    const double lo = d->edges_mrad[2 * j], hi = d->edges_mrad[2 * j + 1];
    if (!std::isfinite(lo) || !std::isfinite(hi) || lo < 0.0 || hi < lo)
      return fail(PRISM_EINVAL, "detector edges must satisfy 0 <= inner <= outer");
    b->lo[j] = (int)p->first_ge(lo * 1e-3);
    b->hi[j] = (int)p->first_ge(hi * 1e-3);
  }
  return PRISM_OK;
}

prism::ProbeOptics probe_optics(const prism_plan* p, const prism_optics* o) {
  prism::ProbeOptics po{};
  po.lam = p->lam;
  po.dq = p->dq;
  po.C1 = o->C1_A;
  po.C3 = o->C3_A;
  po.cell = p->cell;
  po.ktx = p->tilt_k(o->tilt_x_mrad);
  po.kty = p->tilt_k(o->tilt_y_mrad);
  po.sx = p->height * std::tan(o->tilt_x_mrad * 1e-3);
  po.sy = p->height * std::tan(o->tilt_y_mrad * 1e-3);
  po.norm = 1.0;
  return po;
}

// Beams of the set inside the (tilted) probe aperture.
const std::vector<prism::ActiveBeam>* get_active(prism_plan* p, int f, double amax_mrad,
                                                 const std::vector<int32_t>& mn,
                                                 const prism_optics* o) {
  const auto key = std::make_tuple(f, dbits(amax_mrad), dbits(o->alpha_mrad),
                                   dbits(o->tilt_x_mrad), dbits(o->tilt_y_mrad));
  auto it = p->active.find(key);
  if (it != p->active.end()) return &it->second;
  std::vector<prism::ActiveBeam> act;
  for (size_t b = 0; b < mn.size() / 2; ++b)
    if (p->in_aperture((long long)mn[2 * b] * f, (long long)mn[2 * b + 1] * f, o))
      act.push_back(prism::ActiveBeam{(int)b, mn[2 * b], mn[2 * b + 1]});
  return &(p->active[key] = std::move(act));
}

// Per-bin pixel lists of the W x W PRISM window: pixel (v, u) has full-grid
// frequency f * (kx, ky) with (kx, ky) the window's fftfreq indices. Each
// bin's list is padded to whole chunks of kWdListChunk entries.
const prism_plan::PixLists* get_pixlists(prism_plan* p, int w, int f, const prism::DetBins& b) {
  std::string key = std::to_string(w) + ":" + std::to_string(f);
  for (int j = 0; j < b.n; ++j) key += ":" + std::to_string(b.lo[j]) + "-" + std::to_string(b.hi[j]);
  auto it = p->pixlists.find(key);
  if (it != p->pixlists.end()) return &it->second;
  prism_plan::PixLists pl;
  std::memset(&pl.lists, 0, sizeof pl.lists);
  pl.lists.n = b.n;
  const size_t chunk = prism::kWdListChunk;
  for (int j = 0; j < b.n; ++j) {
    pl.lists.off[j] = (int)(pl.pix.size() / chunk);
    for (int v = 0; v < w; ++v) {
      const long long ky = v < w / 2 ? v : v - w;
      for (int u = 0; u < w; ++u) {
        const long long kx = u < w / 2 ? u : u - w;
        const long long k2 = (long long)f * f * (kx * kx + ky * ky);
        if (k2 >= b.lo[j] && k2 < b.hi[j]) pl.pix.push_back((uint16_t)(v * w + u));
      }
    }
    pl.pix.resize((pl.pix.size() + chunk - 1) / chunk * chunk, prism::kNoPix);
  }
  pl.lists.off[b.n] = (int)(pl.pix.size() / chunk);
  return &(p->pixlists[key] = std::move(pl));
}

// ---------------------------------------------------------------- layouts

constexpr size_t kChunkBytes = size_t(1) << 30;  // preferred probe-window bytes per chunk

size_t state_bytes(int n) { return (size_t)n * (n / 2) * sizeof(float2); }

// waves per slice-pass launch: the plan's wave-state bytes per launch
int pref_wave_chunk(const prism_plan* p, int count) {
  const int c = (int)std::max<size_t>(1, p->wave_chunk_bytes / state_bytes(p->n));
  return std::max(1, std::min(c, count));
}

// probes per window-sum group for window side w
int group_of(const prism_plan* p, int w) {
  return p->probe_group > 0 ? p->probe_group : prism::contract_group(w);
}

struct SliceWs {
  float2* twN;
  float2* twH;
  float2* tw2;
  double* thick;
  float2* prop;
  float2* trans;
  int32_t* mn;
  int2* aper;      // multislice: aperture kx interval per full-grid row
  float2* state;
  double* partial;
};

size_t slice_layout(const prism_plan* p, int chunk, int n_beams, int n_det, SliceWs* w, void* base) {
  Carve c(base);
  const int n = p->n;
  w->twN = c.take<float2>(n);
  w->twH = c.take<float2>(n / 2);
  w->tw2 = c.take<float2>(n);
  w->thick = c.take<double>(p->H);
  w->prop = c.take<float2>((size_t)p->H * n);
  w->trans = c.take<float2>((size_t)p->H * n * n);
  w->mn = c.take<int32_t>(2 * (size_t)std::max(n_beams, 0));
  w->aper = c.take<int2>(n_det > 0 ? (size_t)n : 0);
  w->state = c.take<float2>((size_t)chunk * n * (n / 2));
  w->partial = c.take<double>((size_t)chunk * prism::col_tiles(n) * std::max(n_det, 0));
  return c.used + 256;
}

int choose_chunk(const prism_plan* p, int want, int n_beams, int n_det, size_t ws_bytes) {
  SliceWs w;
  for (int c = want; c >= 1; c = (c > 8 ? c * 3 / 4 : c - 1))
    if (slice_layout(p, c, n_beams, n_det, &w, nullptr) <= ws_bytes) return c;
  return 0;
}

// Operand form of the packed window sum for a plan precision.
prism::Prec packed_prec(int prec) {
  return prec == PRISM_PREC_BF16 ? prism::Prec::kBF16
                                 : (prec == PRISM_PREC_FP16 ? prism::Prec::kFP16 : prism::Prec::kF32);
}

// Active beams padded to a whole pair of K blocks.
int padded_beams(int n_act, prism::Prec pk) {
  const int pad = prism::prec_beam_pad(pk);
  return (n_act + pad - 1) / pad * pad;
}

// Probe-step workspace of one sub-batch: requests of one launch class (same
// window side w, group G, operand form), their distinct packed S-matrices
// and detector pixel-list sets, and the per-chunk buffers of `chunk` probes.
struct PackShape {
  int n_act, n_actp, ns;
};
struct PackWs {
  prism::ActiveBeam* act;
  float* scale;       // 16-bit: [n_act] power-of-two beam scales
  float* scale_part;  // 16-bit: [n_act][kScaleSplit] per-block maxima
  uint32_t* s16;      // packed S: [ns^2][n_actp] (re, im), one word (16-bit) or two (FP32)
};
struct ProbeBatchWs {
  float2* twW;
  std::vector<PackWs> packs;
  std::vector<uint16_t*> pix;  // per pixel-list set: bins as lists of window pixels
  std::vector<prism::BinLists*> lists;
  uint32_t* a16;    // packed alpha: [groups][K blocks][2G][32 words]
  int2* origin;     // [chunk]
  float2* window;   // [chunk][w][w]
  double* partial;  // W > 128: [chunk][tiles][PRISM_MAX_DET] detector partials
};

size_t probe_batch_layout(int w, int G, prism::Prec pk, const std::vector<PackShape>& packs,
                    int n_lists, int n_reqs, int chunk, ProbeBatchWs* bw, void* base) {
  Carve c(base);
  bw->twW = c.take<float2>(w);
  bw->packs.resize(packs.size());
  int nblk_max = 1;
  for (size_t k = 0; k < packs.size(); ++k) {
    const PackShape& ps = packs[k];
    PackWs& pw = bw->packs[k];
    pw.act = c.take<prism::ActiveBeam>(ps.n_act);
    pw.scale = pk == prism::Prec::kF32 ? nullptr : c.take<float>(ps.n_act);
    pw.scale_part =
        pk == prism::Prec::kF32 ? nullptr : c.take<float>((size_t)ps.n_act * prism::kScaleSplit);
    pw.s16 = c.take<uint32_t>((size_t)ps.ns * ps.ns * ps.n_actp * prism::prec_words(pk));
    nblk_max = std::max(nblk_max, ps.n_actp / prism::prec_block_beams(pk));
  }
  // per-bin pixel lists (W <= 128), worst case: every bin holds every pixel
  // and a padded last chunk
  bw->pix.resize(n_lists);
  bw->lists.resize(n_lists);
  for (int k = 0; k < n_lists; ++k) {
    bw->pix[k] = c.take<uint16_t>((size_t)PRISM_MAX_DET * ((size_t)w * w + prism::kWdListChunk));
    bw->lists[k] = c.take<prism::BinLists>(1);
  }
  // a chunk's pieces (at most one per request, kMaxSeg at most) each add
  // at most one partial group to the chunk / G whole ones
  const int groups = chunk / G + std::min(prism::kMaxSeg, std::max(n_reqs, 1)) - 1;
  bw->a16 = c.take<uint32_t>((size_t)groups * nblk_max * 2 * G * prism::kC16KB);
  bw->origin = c.take<int2>(chunk);
  bw->window = c.take<float2>((size_t)chunk * w * w);
  bw->partial = prism::window_big(w)
                    ? c.take<double>((size_t)chunk * prism::window_big_tiles(w) * PRISM_MAX_DET)
                    : nullptr;
  return c.used + 256;
}

int pref_probe_chunk(int w, int group) {
  const size_t per = (size_t)w * w * sizeof(float2);
  int c = (int)std::min<size_t>(16384, std::max<size_t>(group, kChunkBytes / per));
  return std::max(group, c / group * group);
}

void* aligned_base(void* ws) {
  const uintptr_t u = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<void*>((u + 255) & ~uintptr_t(255));
}

#define HIP_TRY(expr, where)                       \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

// Kernel launch bracketed by HIP events on its stream when profiling is on.
#define LAUNCH(plan, st, name, expr)                                      \
  do {                                                                  \
    hipEvent_t _a = nullptr, _b = nullptr;                              \
    if ((plan)->prof_on) {                                              \
      _a = (plan)->event();                                             \
      _b = (plan)->event();                                             \
      if (_a) (void)hipEventRecord(_a, st);                                   \
    }                                                                   \
    hipError_t _e = (expr);                                             \
    if (_e != hipSuccess) return hip_fail(_e, name);                    \
    if ((plan)->prof_on && _a && _b) {                                  \
      (void)hipEventRecord(_b, st);                                     \
      (plan)->prof.push_back(ProfRecord{name, _a, _b});                 \
    }                                                                   \
  } while (0)

// Fill twiddles, propagator table and transmission functions of every slice.
int prepare_slices(prism_plan* p, const SliceWs& w, hipStream_t st) {
  const int n = p->n;
  HIP_TRY(hipMemcpyAsync(w.thick, p->thick.data(), p->H * sizeof(double), hipMemcpyHostToDevice, st),
          "copy slice thickness");
  LAUNCH(p, st, "twiddles", prism::launch_twiddles(w.twN, n, st));
  LAUNCH(p, st, "twiddles", prism::launch_twiddles(w.twH, n / 2, st));
  LAUNCH(p, st, "twiddles", prism::launch_twiddles2(w.tw2, n, st));
  LAUNCH(p, st, "prop_lut", prism::launch_prop_lut(w.prop, n, p->H, w.thick, p->lam, p->dq, st));
  LAUNCH(p, st, "transmission", prism::launch_transmission(p->phase, w.trans, (size_t)p->H * n * n, 1.0f / (float)n, st));
  return PRISM_OK;
}

}  // namespace

namespace {

// Output store mode of the public calls: overwrite, or add weight * result.
int out_mode(bool accumulate, double weight, prism::OutAcc* oa) {
  if (accumulate && !std::isfinite(weight)) return fail(PRISM_EINVAL, "weight must be finite");
  *oa = prism::OutAcc{accumulate ? 1 : 0, accumulate ? weight : 1.0};
  return PRISM_OK;
}

// ---------------------------------------------------------------------------
// PRISM probe step (Fig. 1d-f) over a batch of requests. Each request is
// the work of one prism_probe_outputs / prism_probe_cbed call (its own
// specimen, S-matrix, optics, detector and outputs). Requests with the same
// window side, probe group, window tiles, operand form and output kind form
// a launch class: per chunk of probes the window sum and the window
// detector run once over all of the class's requests (one segment each),
// while the S-matrix packing (once per distinct S-matrix and active beam
// set) and the coefficients (per piece) run per request. Every probe group
// lies inside one request and is computed as in a call of its own, so the
// results do not depend on what else is in the batch.

struct Req {
  prism_plan* p;
  int f;
  double amax;
  const float2* S;
  const double* xy;
  int P;
  prism_optics o;
  bool cbed_out;
  prism::DetBins bins;
  double* out;
  float* cbed;
  prism::OutAcc oa;
  const std::vector<prism::ActiveBeam>* act;
  const prism_plan::PixLists* pl;  // detector sums with W <= 128
  prism::ProbeOptics po;           // norm 1: the scale is applied by the window sum
  float out_scale;                 // 1 / (W sqrt(B_A))
  int w, ns, G, tile_div, n_act, n_actp;
  prism::Prec pr;
};

bool same_class(const Req& a, const Req& b) {
  return a.w == b.w && a.G == b.G && a.tile_div == b.tile_div && a.pr == b.pr &&
         a.cbed_out == b.cbed_out;
}
bool same_pack(const Req& a, const Req& b) {
  return a.S == b.S && a.act == b.act && a.pr == b.pr && a.ns == b.ns;
}

// Every check of a probe-step call; buffers are checked only when the call
// is to run (buffers == true) and has probes. d == nullptr: CBED output.
int check_request(prism_plan* p, int f, double amax_mrad, const void* S, size_t S_bytes,
                  const double* xy, int P, const prism_optics* o, const prism_detector* d,
                  double* out, float* cbed, prism::OutAcc oa, bool buffers, Req* r) {
  if (!p) return fail(PRISM_EINVAL, "null plan");
  const std::vector<int32_t>* mn;
  if (int e = beams_checked(p, f, amax_mrad, &mn)) return e;
  if (P < 0) return fail(PRISM_EINVAL, "negative probe count");
  if (int e = check_optics(p, o)) return e;
  if (o->alpha_mrad + std::hypot(o->tilt_x_mrad, o->tilt_y_mrad) > amax_mrad)
    return fail(PRISM_EINVAL, "probe semi-angle plus tilt exceeds the beam set's alpha_max");
  r->cbed_out = d == nullptr;
  std::memset(&r->bins, 0, sizeof r->bins);
  if (!r->cbed_out)
    if (int e = make_bins(p, d, &r->bins)) return e;
  const int n = p->n, w = n / (2 * f);
  if (!prism::window_side_ok(w))
    return fail(PRISM_EINVAL,
                "window side n/(2f) must be a power of two in 8..256 or one of 12, 18, 24, 36, "
                "48, 72, 96, 144, 192");
  const auto* act = get_active(p, f, amax_mrad, *mn, o);
  if (act->empty()) return fail(PRISM_EINVAL, "no beam of the set lies inside the probe aperture");
  if (buffers && P > 0) {
    if (!S || !xy || (r->cbed_out ? !cbed : !out)) return fail(PRISM_EINVAL, "null device buffer");
    if (S_bytes < smatrix_need(p, *mn))
      return fail(PRISM_EINVAL,
                  "S-matrix buffer smaller than prism_smatrix_bytes for this f and alpha_max");
  }
  r->p = p;
  r->f = f;
  r->amax = amax_mrad;
  r->S = static_cast<const float2*>(S);
  r->xy = xy;
  r->P = P;
  r->o = *o;
  r->out = out;
  r->cbed = cbed;
  r->oa = oa;
  r->act = act;
  r->w = w;
  r->ns = n / 2;
  r->G = group_of(p, w);
  r->tile_div = p->tune.window_tile_div;
  r->pr = packed_prec(p->prec);
  r->n_act = (int)act->size();
  r->n_actp = padded_beams(r->n_act, r->pr);
  r->po = probe_optics(p, o);
  r->out_scale = (float)(1.0 / ((double)w * std::sqrt((double)r->n_act)));
  // per-bin pixel lists drive the W <= 128 detector; larger windows bin per element
  r->pl = (prism::window_big(w) || r->cbed_out) ? nullptr : get_pixlists(p, w, f, r->bins);
  return PRISM_OK;
}

// Requests (indices) that run on one workspace fill: their distinct packed
// S-matrices and pixel-list sets.
struct Sub {
  std::vector<int> reqs, pack_of, lists_of;  // per request
  std::vector<int> packs, lists;             // first request of each
  long long probes = 0;
  void add(const std::vector<Req>& rq, int i) {
    const Req& r = rq[i];
    int k = 0;
    while (k < (int)packs.size() && !same_pack(rq[packs[k]], r)) ++k;
    if (k == (int)packs.size()) packs.push_back(i);
    int l = -1;
    if (r.pl) {
      l = 0;
      while (l < (int)lists.size() && rq[lists[l]].pl != r.pl) ++l;
      if (l == (int)lists.size()) lists.push_back(i);
    }
    reqs.push_back(i);
    pack_of.push_back(k);
    lists_of.push_back(l);
    probes += r.P;
  }
  size_t layout(const std::vector<Req>& rq, int chunk, ProbeBatchWs* bw, void* base) const {
    const Req& r0 = rq[reqs[0]];
    std::vector<PackShape> shapes;
    for (int i : packs) shapes.push_back(PackShape{rq[i].n_act, rq[i].n_actp, rq[i].ns});
    return probe_batch_layout(r0.w, r0.G, r0.pr, shapes, (int)lists.size(), (int)reqs.size(),
                              chunk, bw, base);
  }
};

// Probes of one request that one chunk holds: request probes q0 .. q0 + np
// at windows begin .. begin + np of the chunk.
struct Piece {
  int req, sub_idx, q0, np, begin;
};

int run_sub(std::vector<Req>& rq, const Sub& sb, int chunk, void* base, hipStream_t st) {
  ProbeBatchWs bw;
  sb.layout(rq, chunk, &bw, base);
  const Req& r0 = rq[sb.reqs[0]];
  prism_plan* lp = r0.p;  // launches shared by the requests are timed on the first one's plan
  const int w = r0.w, G = r0.G;
  const prism::Prec pr = r0.pr;
  const bool f32 = pr == prism::Prec::kF32, big = prism::window_big(w);
  const size_t w2 = (size_t)w * w;
  LAUNCH(lp, st, "twiddles", prism::launch_twiddles(bw.twW, w, st));
  // host tables come from the plans' caches, whose entries are never
  // rewritten, so the asynchronous copies may read them after the return
  for (size_t l = 0; l < sb.lists.size(); ++l) {
    const prism_plan::PixLists* pl = rq[sb.lists[l]].pl;
    if (!pl->pix.empty())
      HIP_TRY(hipMemcpyAsync(bw.pix[l], pl->pix.data(), pl->pix.size() * sizeof(uint16_t),
                             hipMemcpyHostToDevice, st),
              "copy detector pixel lists");
    HIP_TRY(hipMemcpyAsync(bw.lists[l], &pl->lists, sizeof(prism::BinLists), hipMemcpyHostToDevice,
                           st),
            "copy detector bin offsets");
  }
  for (size_t k = 0; k < sb.packs.size(); ++k) {
    const Req& r = rq[sb.packs[k]];
    const PackWs& pw = bw.packs[k];
    HIP_TRY(hipMemcpyAsync(pw.act, r.act->data(), r.act->size() * sizeof(prism::ActiveBeam),
                           hipMemcpyHostToDevice, st),
            "copy active beams");
    if (!f32)
      LAUNCH(r.p, st, "s16_scale",
             prism::launch_s16_scale(r.S, pw.act, r.n_act, r.ns, pw.scale_part, pw.scale, st));
    LAUNCH(r.p, st, f32 ? "s32_pack" : "s16_pack",
           prism::launch_s16_pack(r.S, pw.act, r.n_act, r.n_actp, r.ns, pw.scale, pw.s16, pr, st));
  }
  std::vector<Piece> pc;
  int used = 0;
  auto flush = [&]() -> int {
    prism::ContractSegs cs{};
    cs.n = (int)pc.size();
    size_t a16_off = 0;
    int g = 0;
    for (size_t k = 0; k < pc.size(); ++k) {
      const Piece& x = pc[k];
      const Req& r = rq[x.req];
      const PackWs& pw = bw.packs[sb.pack_of[x.sub_idx]];
      const int nblk = r.n_actp / prism::prec_block_beams(pr);
      const int ngrp = (x.np + G - 1) / G;
      uint32_t* a16 = bw.a16 + a16_off;
      LAUNCH(r.p, st, f32 ? "alpha" : "alpha16",
             prism::launch_alpha16(r.xy, x.q0, x.np, pw.act, r.n_act, r.n_actp, r.f, r.ns, w, r.po,
                                   pw.scale, G, a16, bw.origin + x.begin, pr, st));
      cs.s[k] = prism::ContractSeg{pw.s16, a16, bw.origin + x.begin, bw.window + x.begin * w2,
                                   r.n_actp * prism::prec_words(pr), r.ns, x.np, g, r.out_scale};
      g += ngrp;
      a16_off += (size_t)ngrp * nblk * 2 * G * prism::kC16KB;
    }
    cs.groups = g;
    LAUNCH(lp, st, f32 ? "contract" : "contract16",
           prism::launch_contract16(cs, w, G, pr, r0.tile_div, st));
    // window FFT, |Psi|^2 and detector sums (or the CBED)
    if (big) {
      for (const Piece& x : pc) {
        const Req& r = rq[x.req];
        float2* win = bw.window + x.begin * w2;
        if (r.cbed_out) {
          LAUNCH(r.p, st, "window_big_cbed",
                 prism::launch_window_big(win, x.np, w, bw.twW, r.f, r.bins, nullptr,
                                          r.cbed + (size_t)x.q0 * w2, r.oa, st));
        } else {
          LAUNCH(r.p, st, "window_big",
                 prism::launch_window_big(win, x.np, w, bw.twW, r.f, r.bins, bw.partial, nullptr,
                                          prism::OutAcc{0, 1.0}, st));
          LAUNCH(r.p, st, "reduce_partials",
                 prism::launch_reduce_partials(bw.partial, x.np, prism::window_big_tiles(w),
                                               r.bins.n, r.out + (size_t)x.q0 * r.bins.n, r.oa,
                                               st));
        }
      }
    } else {
      prism::WindowSegs ws{};
      ws.n = (int)pc.size();
      ws.total = used;
      for (size_t k = 0; k < pc.size(); ++k) {
        const Piece& x = pc[k];
        const Req& r = rq[x.req];
        const int l = sb.lists_of[x.sub_idx];
        ws.s[k] = prism::WindowSeg{l >= 0 ? bw.pix[l] : nullptr, l >= 0 ? bw.lists[l] : nullptr,
                                   r.cbed_out ? nullptr : r.out + (size_t)x.q0 * r.bins.n,
                                   r.cbed_out ? r.cbed + (size_t)x.q0 * w2 : nullptr, r.oa,
                                   x.begin};
      }
      if (r0.cbed_out) {
        LAUNCH(lp, st, "window_cbed", prism::launch_window_cbed(bw.window, ws, w, bw.twW, st));
      } else {
        LAUNCH(lp, st, "window_detect", prism::launch_window_detect(bw.window, ws, w, bw.twW, st));
      }
    }
    pc.clear();
    used = 0;
    return PRISM_OK;
  };
  for (size_t i = 0; i < sb.reqs.size(); ++i) {
    const Req& r = rq[sb.reqs[i]];
    for (int q = 0; q < r.P;) {
      const int take = std::min(r.P - q, chunk - used);
      pc.push_back(Piece{sb.reqs[i], (int)i, q, take, used});
      used += take;
      q += take;
      if (used == chunk || (int)pc.size() == prism::kMaxSeg)
        if (int e = flush()) return e;
    }
  }
  if (!pc.empty())
    if (int e = flush()) return e;
  return PRISM_OK;
}

// The requests of one launch class, in order, in as few workspace fills as
// the workspace allows.
int run_class(std::vector<Req>& rq, const std::vector<int>& members, void* ws, size_t ws_bytes,
              hipStream_t st) {
  void* base = aligned_base(ws);
  const int G = rq[members[0]].G;
  const int pref = pref_probe_chunk(rq[members[0]].w, G);
  auto chunk_for = [&](long long probes) {
    return (int)std::max<long long>(G, std::min<long long>(pref, (probes + G - 1) / G * G));
  };
  ProbeBatchWs probe_ws;
  size_t i = 0;
  while (i < members.size()) {
    Sub sb;
    int chunk = 0;
    for (size_t j = i; j < members.size(); ++j) {
      Sub t = sb;
      t.add(rq, members[j]);
      const int c = chunk_for(t.probes);
      if (t.layout(rq, c, &probe_ws, nullptr) > ws_bytes) break;
      sb = std::move(t);
      chunk = c;
    }
    if (sb.reqs.empty()) {
      // the next request alone, on fewer probes per chunk
      sb.add(rq, members[i]);
      chunk = chunk_for(sb.probes);
      while (chunk >= G && sb.layout(rq, chunk, &probe_ws, nullptr) > ws_bytes)
        chunk = chunk > 8 * G ? (chunk * 3 / 4) / G * G : chunk - G;
      if (chunk < G) return fail(PRISM_ENOSPACE, "workspace smaller than the probe-step minimum");
    }
    if (int e = run_sub(rq, sb, chunk, base, st)) return e;
    i += sb.reqs.size();
  }
  return PRISM_OK;
}

// Launch classes in order of first appearance; requests without probes run
// nothing.
int run_batch(std::vector<Req>& rq, void* ws, size_t ws_bytes, hipStream_t st) {
  std::vector<std::vector<int>> classes;
  for (int i = 0; i < (int)rq.size(); ++i) {
    if (rq[i].P == 0) continue;
    size_t c = 0;
    while (c < classes.size() && !same_class(rq[classes[c][0]], rq[i])) ++c;
    if (c == classes.size()) classes.emplace_back();
    classes[c].push_back(i);
  }
  if (classes.empty()) return PRISM_OK;
  if (!ws) return fail(PRISM_EINVAL, "null workspace");
  for (const auto& members : classes)
    if (int e = run_class(rq, members, ws, ws_bytes, st)) return e;
  return PRISM_OK;
}

int probe_step(prism_plan* p, int f, double amax_mrad, const void* S, size_t S_bytes,
               const double* xy, int P, const prism_optics* o, const prism_detector* d,
               double* out, float* cbed, prism::OutAcc oa, void* ws, size_t ws_bytes,
               void* stream) {
  std::vector<Req> rq(1);
  if (int e = check_request(p, f, amax_mrad, S, S_bytes, xy, P, o, d, out, cbed, oa, true, &rq[0]))
    return e;
  return run_batch(rq, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

// Multislice STEM (Fig. 1a-c): one full-grid wave per probe, H slice steps,
// detector sums of |Psi|^2; oa as in probe_step.
int multislice_step(prism_plan* p, const double* xy, int P, const prism_optics* o,
                    const prism_detector* d, double* out, prism::OutAcc oa, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!p) return fail(PRISM_EINVAL, "null plan");
  if (P < 0) return fail(PRISM_EINVAL, "negative probe count");
  if (int r = check_optics(p, o)) return r;
  prism::DetBins bins;
  if (int r = make_bins(p, d, &bins)) return r;
  if (P == 0) return PRISM_OK;
  if (!xy || !out || !ws) return fail(PRISM_EINVAL, "null device buffer");
  if (!p->phase) return fail(PRISM_ENOTREADY, "potential slices not set");
  const int n = p->n;
  void* base = aligned_base(ws);
  const int chunk = choose_chunk(p, pref_wave_chunk(p, P), 0, bins.n, ws_bytes);
  if (chunk < 1) return fail(PRISM_ENOSPACE, "workspace smaller than the multislice minimum");
  SliceWs w;
  slice_layout(p, chunk, 0, bins.n, &w, base);
  prism::ProbeOptics po = probe_optics(p, o);
  const auto akey =
      std::make_tuple(dbits(o->alpha_mrad), dbits(o->tilt_x_mrad), dbits(o->tilt_y_mrad));
  auto ait = p->aper_rows.find(akey);
  if (ait == p->aper_rows.end()) {
    prism_plan::AperRows ar;
    ar.count = aperture_rows(p, o, &ar.rows);
    ait = p->aper_rows.emplace(akey, std::move(ar)).first;
  }
  const std::vector<int32_t>& rows = ait->second.rows;
  const long long n_ap = ait->second.count;
  if (n_ap < 1) return fail(PRISM_EINVAL, "the probe aperture holds no grid frequency");
  po.norm = 1.0 / std::sqrt((double)n_ap);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int r = prepare_slices(p, w, st)) return r;
  HIP_TRY(hipMemcpyAsync(w.aper, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                         st),
          "copy aperture rows");
  const int tiles = prism::col_tiles(n);
  for (int p0 = 0; p0 < P; p0 += chunk) {
    const int np = std::min(chunk, P - p0);
    LAUNCH(p, st, "probe_init", prism::launch_probe_init(w.state, xy, p0, np, n, po, w.aper, w.twN, st));
    for (int s = 0; s < p->H; ++s) {
      LAUNCH(p, st, "row_pass", prism::launch_row_pass(w.state, np, n, w.trans + (size_t)s * n * n, w.twN, w.tw2, p->tune, st));
      if (s + 1 < p->H) {
        LAUNCH(p, st, "col_pass", prism::launch_col_pass(w.state, np, n, w.prop + (size_t)s * n, w.twN, w.tw2, p->tune, st));
      } else {
        LAUNCH(p, st, "col_detect", prism::launch_col_detect(w.state, np, n, w.prop + (size_t)s * n, w.twN, bins,
                                         w.partial, st));
      }
    }
    LAUNCH(p, st, "reduce_partials",
           prism::launch_reduce_partials(w.partial, np, tiles, bins.n, out + (size_t)p0 * bins.n,
                                         oa, st));
  }
  return PRISM_OK;
}


}  // namespace

// =========================================================================
// C ABI
// =========================================================================

extern "C" {

const char* prism_last_error(void) { return g_err.c_str(); }

int prism_plan_create(prism_plan** out, const prism_geometry* g) {
  if (!out || !g) return fail(PRISM_EINVAL, "null argument");
  *out = nullptr;
  // grids 2^k, 3 * 2^k or 9 * 2^k (the LDS transforms have radices 2, 4, 8,
  // 3 and 9)
  const bool grid_ok = is_pow2(g->n) || (g->n % 3 == 0 && is_pow2(g->n / 3)) ||
                       (g->n % 9 == 0 && is_pow2(g->n / 9));
  if (!grid_ok || g->n < 128 || g->n > 2048)
    return fail(PRISM_EINVAL, "n must be 2^k, 3 * 2^k or 9 * 2^k in [128, 2048]");
  if (!(g->cell_A > 0.0) || !std::isfinite(g->cell_A)) return fail(PRISM_EINVAL, "cell must be > 0");
  if (!(g->energy_keV > 0.0) || !std::isfinite(g->energy_keV))
    return fail(PRISM_EINVAL, "energy must be > 0");
  if (g->n_slices < 1 || !g->slice_thickness_A) return fail(PRISM_EINVAL, "need >= 1 slice");
  for (int i = 0; i < g->n_slices; ++i)
    if (!(g->slice_thickness_A[i] > 0.0) || !std::isfinite(g->slice_thickness_A[i]))
      return fail(PRISM_EINVAL, "slice thickness must be > 0");
  auto* p = new prism_plan();
  p->n = g->n;
  p->cell = g->cell_A;
  p->energy = g->energy_keV;
  p->lam = kHcKeVA / std::sqrt(g->energy_keV * (g->energy_keV + 2.0 * kMec2KeV));
  p->dq = 1.0 / g->cell_A;
  p->H = g->n_slices;
  p->thick.assign(g->slice_thickness_A, g->slice_thickness_A + g->n_slices);
  for (double t : p->thick) p->height += t;
  *out = p;
  return PRISM_OK;
}

void prism_plan_destroy(prism_plan* plan) { delete plan; }

int prism_wavelength(const prism_plan* p, double* lam) {
  if (!p || !lam) return fail(PRISM_EINVAL, "null argument");
  *lam = p->lam;
  return PRISM_OK;
}

int prism_alpha_max(const prism_plan* p, int f, double alpha_mrad, double* alpha_max_mrad) {
  if (!p || !alpha_max_mrad) return fail(PRISM_EINVAL, "null argument");
  if (int r = check_f(p, f)) return r;
  if (!(alpha_mrad > 0.0) || !std::isfinite(alpha_mrad))
    return fail(PRISM_EINVAL, "alpha_mrad must be positive and finite");
  // one beam-spacing margin beyond the largest probe semi-angle: the
  // interpolated beam pitch is f dq, i.e. f lambda dq in angle
  *alpha_max_mrad = alpha_mrad + (double)f * (p->lam * p->dq) * 1e3;
  return PRISM_OK;
}

int prism_active_beam_count(const prism_plan* cp, int f, double amax_mrad,
                            const prism_optics* o, int* n_active) {
  if (!n_active) return fail(PRISM_EINVAL, "null argument");
  prism_plan* p = const_cast<prism_plan*>(cp);
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  if (int r = check_optics(p, o)) return r;
  *n_active = (int)get_active(p, f, amax_mrad, *mn, o)->size();
  return PRISM_OK;
}

int prism_beam_count(const prism_plan* p, int f, double amax_mrad, int* n_beams) {
  if (!n_beams) return fail(PRISM_EINVAL, "null argument");
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  *n_beams = (int)(mn->size() / 2);
  return PRISM_OK;
}

int prism_beams(const prism_plan* p, int f, double amax_mrad, int32_t* out, int capacity) {
  if (!out || capacity < 0) return fail(PRISM_EINVAL, "null argument");
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  const size_t cnt = std::min(mn->size() / 2, (size_t)capacity);
  std::memcpy(out, mn->data(), cnt * 2 * sizeof(int32_t));
  return PRISM_OK;
}

int prism_smatrix_bytes(const prism_plan* p, int f, double amax_mrad, size_t* bytes) {
  if (!bytes) return fail(PRISM_EINVAL, "null argument");
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  *bytes = smatrix_need(p, *mn);
  return PRISM_OK;
}

int prism_build_workspace_bytes(const prism_plan* p, int f, double amax_mrad, size_t* pref,
                                size_t* minimum) {
  if (!pref || !minimum) return fail(PRISM_EINVAL, "null argument");
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  const int B = (int)(mn->size() / 2);
  SliceWs w;
  *pref = slice_layout(p, pref_wave_chunk(p, B), B, 0, &w, nullptr);
  *minimum = slice_layout(p, 1, B, 0, &w, nullptr);
  return PRISM_OK;
}

int prism_multislice_workspace_bytes(const prism_plan* p, int n_det, size_t* pref,
                                     size_t* minimum) {
  if (!p || !pref || !minimum) return fail(PRISM_EINVAL, "null argument");
  if (n_det < 1 || n_det > PRISM_MAX_DET) return fail(PRISM_EINVAL, "n_det out of range");
  SliceWs w;
  *pref = slice_layout(p, pref_wave_chunk(p, 1 << 20), 0, n_det, &w, nullptr);
  *minimum = slice_layout(p, 1, 0, n_det, &w, nullptr);
  return PRISM_OK;
}

int prism_probe_class(const prism_plan* p, int f, unsigned long long* key) {
  if (!p || !key) return fail(PRISM_EINVAL, "null argument");
  if (int r = check_f(p, f)) return r;
  const int w = p->n / (2 * f);
  if (!prism::window_side_ok(w))
    return fail(PRISM_EINVAL,
                "window side n/(2f) must be a power of two in 8..256 or one of 12, 18, 24, 36, "
                "48, 72, 96, 144, 192");
  *key = (unsigned long long)w | (unsigned long long)group_of(p, w) << 16 |
         (unsigned long long)p->tune.window_tile_div << 32 |
         (unsigned long long)packed_prec(p->prec) << 48;
  return PRISM_OK;
}

int prism_probe_group(const prism_plan* p, int f, int* group, int* tx, int* ty) {
  if (!p || !group || !tx || !ty) return fail(PRISM_EINVAL, "null argument");
  if (int r = check_f(p, f)) return r;
  const int w = p->n / (2 * f);
  *group = group_of(p, w);
  *tx = 8;
  *ty = *group / 8;
  if (*group == 16) *tx = *ty = 4;
  return PRISM_OK;
}

int prism_probe_order(const prism_plan* p, int f, const double* xy, int P, int32_t* perm) {
  if (!p || (P > 0 && (!xy || !perm))) return fail(PRISM_EINVAL, "null argument");
  if (P < 0) return fail(PRISM_EINVAL, "negative probe count");
  if (int r = check_f(p, f)) return r;
  const int ns = p->n / 2, w = ns / f;
  const int cell = std::max(1, std::min(16, w / 8));
  const double dxs = p->cell / ns;
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)P);
  for (int i = 0; i < P; ++i) {
    // window centre pixel of Eq. RegionBounds, as the coefficient kernel takes it
    long long cx = (long long)std::floor(xy[2 * i] / dxs + 0.5) % ns;
    long long cy = (long long)std::floor(xy[2 * i + 1] / dxs + 0.5) % ns;
    if (cx < 0) cx += ns;
    if (cy < 0) cy += ns;
    const uint32_t gx = (uint32_t)(cx / cell), gy = (uint32_t)(cy / cell);
    uint64_t m = 0;
    for (int b = 0; b < 16; ++b)
      m |= (uint64_t)((gx >> b) & 1u) << (2 * b) | (uint64_t)((gy >> b) & 1u) << (2 * b + 1);
    key[(size_t)i] = {m, i};
  }
  std::sort(key.begin(), key.end());  // ties keep the input order (second member)
  for (int i = 0; i < P; ++i) perm[i] = key[(size_t)i].second;
  return PRISM_OK;
}

int prism_probe_workspace_bytes(const prism_plan* cp, int f, double amax_mrad,
                                const prism_optics* o, size_t* pref, size_t* minimum) {
  if (!pref || !minimum) return fail(PRISM_EINVAL, "null argument");
  prism_plan* p = const_cast<prism_plan*>(cp);
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  if (int r = check_optics(p, o)) return r;
  const int w = p->n / (2 * f);
  if (!prism::window_side_ok(w))
    return fail(PRISM_EINVAL,
                "window side n/(2f) must be a power of two in 8..256 or one of 12, 18, 24, 36, "
                "48, 72, 96, 144, 192");
  const auto* act = get_active(p, f, amax_mrad, *mn, o);
  const int G = group_of(p, w);
  const prism::Prec pk = packed_prec(p->prec);
  const int n_act = (int)act->size();
  const std::vector<PackShape> shapes{PackShape{n_act, padded_beams(n_act, pk), p->n / 2}};
  const int n_lists = prism::window_big(w) ? 0 : 1;
  ProbeBatchWs bw;
  *pref = probe_batch_layout(w, G, pk, shapes, n_lists, 1, pref_probe_chunk(w, G), &bw, nullptr);
  *minimum = probe_batch_layout(w, G, pk, shapes, n_lists, 1, G, &bw, nullptr);
  return PRISM_OK;
}

int prism_set_tuning(prism_plan* p, const prism_tuning* t) {
  if (!p || !t) return fail(PRISM_EINVAL, "null argument");
  auto pow2_in = [](int v, int hi) { return v == 0 || (v >= 1 && v <= hi && (v & (v - 1)) == 0); };
  if (!pow2_in(t->row_iters, 64) || !pow2_in(t->col_iters, 64))
    return fail(PRISM_EINVAL, "row_iters and col_iters must be 0 or powers of two up to 64");
  if (t->row_min_groups < 0 || t->row_min_groups > (1 << 20) || t->col_min_groups < 0 ||
      t->col_min_groups > (1 << 20))
    return fail(PRISM_EINVAL, "row_min_groups and col_min_groups must be in [0, 2^20]");
  if (t->wave_chunk_mib != 0 && (t->wave_chunk_mib < 16 || t->wave_chunk_mib > 65536))
    return fail(PRISM_EINVAL, "wave_chunk_mib must be 0 or in [16, 65536]");
  if (t->probe_group != 0 && t->probe_group != 16 && t->probe_group != 32 && t->probe_group != 64)
    return fail(PRISM_EINVAL, "probe_group must be 0, 16, 32 or 64");
  if (t->window_tile_div < 0 || t->window_tile_div > 64)
    return fail(PRISM_EINVAL, "window_tile_div must be in [0, 64]");
  const prism::LaunchTuning def;
  p->tune.row_iters = t->row_iters ? t->row_iters : def.row_iters;
  p->tune.row_min_wg = t->row_min_groups ? t->row_min_groups : def.row_min_wg;
  p->tune.col_iters = t->col_iters ? t->col_iters : def.col_iters;
  p->tune.col_min_wg = t->col_min_groups ? t->col_min_groups : def.col_min_wg;
  p->tune.window_tile_div = t->window_tile_div ? t->window_tile_div : def.window_tile_div;
  p->wave_chunk_bytes = (size_t)(t->wave_chunk_mib ? t->wave_chunk_mib : 256) << 20;
  p->probe_group = t->probe_group;
  return PRISM_OK;
}

int prism_get_tuning(const prism_plan* p, prism_tuning* t) {
  if (!p || !t) return fail(PRISM_EINVAL, "null argument");
  t->row_iters = p->tune.row_iters;
  t->row_min_groups = p->tune.row_min_wg;
  t->col_iters = p->tune.col_iters;
  t->col_min_groups = p->tune.col_min_wg;
  t->wave_chunk_mib = (int)(p->wave_chunk_bytes >> 20);
  t->probe_group = p->probe_group;
  t->window_tile_div = p->tune.window_tile_div;
  return PRISM_OK;
}

int prism_profile_enable(prism_plan* p, int enable) {
  if (!p) return fail(PRISM_EINVAL, "null plan");
  p->prof_on = enable != 0;
  return PRISM_OK;
}

int prism_profile_report(prism_plan* p, char* buf, size_t len) {
  if (!p || !buf || len == 0) return fail(PRISM_EINVAL, "null argument");
  struct Acc {
    int count = 0;
    double total = 0, mn = 1e300, mx = 0;
  };
  std::map<std::string, Acc> acc;
  int status = PRISM_OK;
  for (auto& r : p->prof) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess && status == PRISM_OK) status = hip_fail(e, "profile events");
    Acc& a = acc[r.name];
    a.count++;
    a.total += ms;
    a.mn = std::min(a.mn, (double)ms);
    a.mx = std::max(a.mx, (double)ms);
    p->ev_pool.push_back(r.start);
    p->ev_pool.push_back(r.stop);
  }
  p->prof.clear();
  std::string text;
  char line[256];
  for (auto& kv : acc) {
    std::snprintf(line, sizeof line, "%s %d %.6f %.6f %.6f\n", kv.first.c_str(), kv.second.count,
                  kv.second.total, kv.second.mn, kv.second.mx);
    text += line;
  }
  if (text.size() + 1 > len) return fail(PRISM_ENOSPACE, "profile report buffer too small");
  std::memcpy(buf, text.c_str(), text.size() + 1);
  return status;
}

int prism_set_probe_precision(prism_plan* p, int precision) {
  if (!p) return fail(PRISM_EINVAL, "null plan");
  if (precision != PRISM_PREC_FP32 && precision != PRISM_PREC_BF16 && precision != PRISM_PREC_FP16)
    return fail(PRISM_EINVAL, "precision must be PRISM_PREC_FP32, _BF16 or _FP16");
  p->prec = precision;
  return PRISM_OK;
}

int prism_set_potential_slices(prism_plan* p, const float* phase_dev) {
  if (!p || !phase_dev) return fail(PRISM_EINVAL, "null argument");
  p->phase = phase_dev;
  return PRISM_OK;
}

#ifndef PRISM_BUILD_STREAMS
#define PRISM_BUILD_STREAMS 2
#endif

int prism_build_smatrix(prism_plan* p, int f, double amax_mrad, void* S, size_t S_bytes, void* ws,
                        size_t ws_bytes, void* stream) {
  const std::vector<int32_t>* mn;
  if (int r = beams_checked(p, f, amax_mrad, &mn)) return r;
  if (!S || !ws) return fail(PRISM_EINVAL, "null device buffer");
  if (S_bytes < smatrix_need(p, *mn))
    return fail(PRISM_EINVAL, "S-matrix buffer smaller than prism_smatrix_bytes for this f and alpha_max");
  if (!p->phase) return fail(PRISM_ENOTREADY, "potential slices not set");
  const int n = p->n, B = (int)(mn->size() / 2);
  void* base = aligned_base(ws);
  const int chunk = choose_chunk(p, pref_wave_chunk(p, B), B, 0, ws_bytes);
  if (chunk < 1) return fail(PRISM_ENOSPACE, "workspace smaller than the build minimum");
  SliceWs w;
  slice_layout(p, chunk, B, 0, &w, base);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int r = prepare_slices(p, w, st)) return r;
  HIP_TRY(hipMemcpyAsync(w.mn, mn->data(), mn->size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
          "copy beam list");
  float2* Sout = static_cast<float2*>(S);
  const size_t splane = (size_t)(n / 2) * (n / 2);
  // Small builds (at most two chunks of beams, so single launches leave the
  // GPU partly idle) run in two lanes: the state buffer is split in two and
  // alternate beam groups run on the caller's stream and on the plan's
  // second stream, so that one group's VALU-heavy row pass overlaps the
  // other's memory-bound column pass. Larger builds keep one lane, where
  // every launch fills the GPU and kernel timings stay exclusive.
  const int lanes =
      (PRISM_BUILD_STREAMS > 1 && chunk >= 2 && B > chunk / 2 && B <= 2 * chunk) ? 2 : 1;
  const int sub = chunk / lanes;
  hipStream_t ls[2] = {st, st};
  if (lanes == 2) {
    if (!p->aux) HIP_TRY(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking), "create build stream");
    if (!p->fork_ev) HIP_TRY(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming), "create event");
    if (!p->join_ev) HIP_TRY(hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming), "create event");
    ls[1] = p->aux;
    HIP_TRY(hipEventRecord(p->fork_ev, st), "fork build stream");
    HIP_TRY(hipStreamWaitEvent(p->aux, p->fork_ev, 0), "fork build stream");
  }
  int g = 0;
  for (int b0 = 0; b0 < B; b0 += sub, ++g) {
    const int nb = std::min(sub, B - b0);
    hipStream_t sg = ls[g % lanes];
    float2* state = w.state + (size_t)(g % lanes) * sub * n * (n / 2);
    LAUNCH(p, sg, "beam_init", prism::launch_beam_init(state, w.mn, b0, nb, n, f, w.twN, sg));
    for (int s = 0; s < p->H; ++s) {
      LAUNCH(p, sg, "row_pass", prism::launch_row_pass(state, nb, n, w.trans + (size_t)s * n * n, w.twN, w.tw2, p->tune, sg));
      LAUNCH(p, sg, "col_pass", prism::launch_col_pass(state, nb, n, w.prop + (size_t)s * n, w.twN, w.tw2, p->tune, sg));
    }
    LAUNCH(p, sg, "extract", prism::launch_extract(state, nb, n, Sout + (size_t)b0 * splane, w.twH, sg));
  }
  if (lanes == 2) {
    HIP_TRY(hipEventRecord(p->join_ev, p->aux), "join build stream");
    HIP_TRY(hipStreamWaitEvent(st, p->join_ev, 0), "join build stream");
  }
  return PRISM_OK;
}

int prism_multislice_outputs(prism_plan* p, const double* xy, int P, const prism_optics* o,
                             const prism_detector* d, double* out, void* ws, size_t ws_bytes,
                             void* stream) {
  return multislice_step(p, xy, P, o, d, out, prism::OutAcc{0, 1.0}, ws, ws_bytes, stream);
}

int prism_multislice_outputs_accumulate(prism_plan* p, const double* xy, int P,
                                        const prism_optics* o, const prism_detector* d,
                                        double weight, double* out, void* ws, size_t ws_bytes,
                                        void* stream) {
  prism::OutAcc oa;
  if (int r = out_mode(true, weight, &oa)) return r;
  return multislice_step(p, xy, P, o, d, out, oa, ws, ws_bytes, stream);
}

int prism_probe_outputs(prism_plan* p, int f, double amax_mrad, const void* S, size_t S_bytes,
                        const double* xy, int P, const prism_optics* o, const prism_detector* d,
                        double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!d) return fail(PRISM_EINVAL, "null detector");
  return probe_step(p, f, amax_mrad, S, S_bytes, xy, P, o, d, out, nullptr,
                    prism::OutAcc{0, 1.0}, ws, ws_bytes, stream);
}

int prism_probe_outputs_accumulate(prism_plan* p, int f, double amax_mrad, const void* S,
                                   size_t S_bytes, const double* xy, int P, const prism_optics* o,
                                   const prism_detector* d, double weight, double* out, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!d) return fail(PRISM_EINVAL, "null detector");
  prism::OutAcc oa;
  if (int r = out_mode(true, weight, &oa)) return r;
  return probe_step(p, f, amax_mrad, S, S_bytes, xy, P, o, d, out, nullptr, oa, ws, ws_bytes,
                    stream);
}

int prism_probe_cbed(prism_plan* p, int f, double amax_mrad, const void* S, size_t S_bytes,
                     const double* xy, int P, const prism_optics* o, float* cbed, void* ws,
                     size_t ws_bytes, void* stream) {
  return probe_step(p, f, amax_mrad, S, S_bytes, xy, P, o, nullptr, nullptr, cbed,
                    prism::OutAcc{0, 1.0}, ws, ws_bytes, stream);
}

int prism_probe_cbed_accumulate(prism_plan* p, int f, double amax_mrad, const void* S,
                                size_t S_bytes, const double* xy, int P, const prism_optics* o,
                                double weight,
                                float* cbed, void* ws, size_t ws_bytes, void* stream) {
  prism::OutAcc oa;
  if (int r = out_mode(true, weight, &oa)) return r;
  return probe_step(p, f, amax_mrad, S, S_bytes, xy, P, o, nullptr, nullptr, cbed, oa, ws,
                    ws_bytes, stream);
}

}  // extern "C"

namespace {

// Checked requests of a batch call (buffers: also the device pointers).
int check_batch(const prism_probe_request* rqs, int count, bool buffers, std::vector<Req>* rq) {
  if (count < 0) return fail(PRISM_EINVAL, "negative request count");
  if (count > 0 && !rqs) return fail(PRISM_EINVAL, "null requests");
  rq->resize(count);
  for (int i = 0; i < count; ++i) {
    const prism_probe_request& q = rqs[i];
    prism::OutAcc oa;
    int e = out_mode(q.accumulate != 0, q.weight, &oa);
    if (!e)
      e = check_request(q.plan, q.f, q.alpha_max_mrad, q.smatrix_dev, q.smatrix_bytes,
                        q.probe_xy_dev, q.n_probes, q.optics, q.detector, q.out_dev, q.cbed_dev,
                        oa, buffers, &(*rq)[i]);
    if (e) return fail(e, "request " + std::to_string(i) + ": " + g_err);
  }
  return PRISM_OK;
}

}  // namespace

extern "C" {

int prism_probe_batch_workspace_bytes(const prism_probe_request* requests, int count,
                                      size_t* pref, size_t* minimum) {
  if (!pref || !minimum) return fail(PRISM_EINVAL, "null argument");
  std::vector<Req> rq;
  if (int e = check_batch(requests, count, false, &rq)) return e;
  *pref = 0;
  *minimum = 0;
  ProbeBatchWs bw;
  std::vector<bool> done(rq.size(), false);
  for (size_t i = 0; i < rq.size(); ++i) {
    Sub one;
    one.add(rq, (int)i);
    *minimum = std::max(*minimum, one.layout(rq, rq[i].G, &bw, nullptr));
    if (done[i]) continue;
    Sub cls;  // every request of i's launch class
    for (size_t j = i; j < rq.size(); ++j)
      if (!done[j] && same_class(rq[i], rq[j])) {
        cls.add(rq, (int)j);
        done[j] = true;
      }
    const long long G = rq[i].G;
    const int chunk = (int)std::max<long long>(
        G, std::min<long long>(pref_probe_chunk(rq[i].w, rq[i].G), (cls.probes + G - 1) / G * G));
    *pref = std::max(*pref, cls.layout(rq, chunk, &bw, nullptr));
  }
  return PRISM_OK;
}

int prism_probe_batch(const prism_probe_request* requests, int count, void* ws, size_t ws_bytes,
                      void* stream) {
  std::vector<Req> rq;
  if (int e = check_batch(requests, count, true, &rq)) return e;
  return run_batch(rq, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched S-matrix build over several specimens.

namespace {

// Specimens whose waves can share launches: same grid, cell and energy, and
// slice thicknesses that agree on their common slices (so one propagator
// table serves all of them). Members are sorted by slice count, largest
// first: the waves still running at slice s are then a prefix.
struct BatchGroup {
  std::vector<int> items;  // indices into the caller's item list
  const prism_plan* ref;   // member with the most slices (its thicknesses)
};

bool same_medium(const prism_plan* a, const prism_plan* b) {
  if (a->n != b->n || dbits(a->cell) != dbits(b->cell) || dbits(a->energy) != dbits(b->energy))
    return false;
  const int h = std::min(a->H, b->H);
  for (int s = 0; s < h; ++s)
    if (dbits(a->thick[s]) != dbits(b->thick[s])) return false;
  return true;
}

// Members whose own chunks are full gain nothing from sharing launches: an
// item with at least kAloneChunks batched launches' worth of beams is built
// on its own (its plan's launch shapes, no per-wave transmission table, no
// members dropping out of shared launches); the others share launches.
constexpr int kAloneChunks = 4;

int batch_pref_chunk(int n, int total);

bool builds_alone(const prism_build_item& it) {
  const int B = (int)(it.plan->beams.at({it.f, dbits(it.alpha_max_mrad)}).size() / 2);
  return B >= kAloneChunks * batch_pref_chunk(it.plan->n, 1 << 30);
}

// Items that share launches, grouped by medium (checked first); *alone
// receives the others.
int batch_groups(const prism_build_item* items, int count, std::vector<BatchGroup>* groups,
                 std::vector<int>* alone) {
  groups->clear();
  alone->clear();
  for (int i = 0; i < count; ++i) {
    const prism_plan* p = items[i].plan;
    if (!p) return fail(PRISM_EINVAL, "batch item " + std::to_string(i) + ": null plan");
    const std::vector<int32_t>* mn;
    if (int r = beams_checked(p, items[i].f, items[i].alpha_max_mrad, &mn))
      return fail(r, "batch item " + std::to_string(i) + ": " + g_err);
    if (builds_alone(items[i])) {
      alone->push_back(i);
      continue;
    }
    BatchGroup* g = nullptr;
    for (auto& cand : *groups) {
      bool ok = true;
      for (int j : cand.items) ok = ok && same_medium(items[j].plan, p);
      if (ok) {
        g = &cand;
        break;
      }
    }
    if (!g) {
      groups->push_back(BatchGroup{{}, p});
      g = &groups->back();
    }
    g->items.push_back(i);
    if (p->H > g->ref->H) g->ref = p;
  }
  for (auto& g : *groups)
    std::stable_sort(g.items.begin(), g.items.end(),
                     [&](int a, int b) { return items[a].plan->H > items[b].plan->H; });
  return PRISM_OK;
}

struct BatchWs {
  float2* twN;
  float2* twH;
  float2* tw2;
  double* thick;
  float2* prop;
  float2* trans;          // every member's slices, member after member
  int32_t* mn;            // every member's beam list
  const float2** wtab;    // per-wave transmission base of the current chunk
  float2* state;
};

int item_beams(const prism_build_item& it) {
  return (int)(it.plan->beams.at({it.f, dbits(it.alpha_max_mrad)}).size() / 2);
}

size_t batch_layout(const prism_build_item* items, const BatchGroup& g, int chunk, BatchWs* w,
                    void* base) {
  Carve c(base);
  const int n = g.ref->n;
  size_t slices = 0, beams = 0;
  for (int i : g.items) {
    slices += items[i].plan->H;
    beams += item_beams(items[i]);
  }
  w->twN = c.take<float2>(n);
  w->twH = c.take<float2>(n / 2);
  w->tw2 = c.take<float2>(n);
  w->thick = c.take<double>(g.ref->H);
  w->prop = c.take<float2>((size_t)g.ref->H * n);
  w->trans = c.take<float2>(slices * n * n);
  w->mn = c.take<int32_t>(2 * beams);
  w->wtab = c.take<const float2*>(chunk);
  w->state = c.take<float2>((size_t)chunk * n * (n / 2));
  return c.used + 256;
}

int batch_total_waves(const prism_build_item* items, const BatchGroup& g) {
  int t = 0;
  for (int i : g.items) t += item_beams(items[i]);
  return t;
}

#ifndef PRISM_BATCH_CHUNK_SHIFT
#define PRISM_BATCH_CHUNK_SHIFT 28  // wave state per batched launch: 2^shift bytes at most
#endif
int batch_pref_chunk(int n, int total) {
  const size_t cap = (size_t(1) << PRISM_BATCH_CHUNK_SHIFT) / state_bytes(n);
  return (int)std::max<size_t>(1, std::min<size_t>(cap, (size_t)total));
}

int batch_build_group(const prism_build_item* items, const BatchGroup& g, void* ws,
                      size_t ws_bytes, hipStream_t st) {
  prism_plan* lead = items[g.items.front()].plan;
  const int n = g.ref->n, total = batch_total_waves(items, g);
  BatchWs w;
  int chunk = batch_pref_chunk(n, total);
  while (chunk >= 1 && batch_layout(items, g, chunk, &w, nullptr) > ws_bytes)
    chunk = chunk > 8 ? chunk * 3 / 4 : chunk - 1;
  if (chunk < 1) return fail(PRISM_ENOSPACE, "workspace smaller than the batched build minimum");
  batch_layout(items, g, chunk, &w, aligned_base(ws));
  prism_plan* p = lead;  // profiling records go to the group's first plan
  HIP_TRY(hipMemcpyAsync(w.thick, g.ref->thick.data(), g.ref->H * sizeof(double),
                         hipMemcpyHostToDevice, st),
          "copy slice thickness");
  LAUNCH(p, st, "twiddles", prism::launch_twiddles(w.twN, n, st));
  LAUNCH(p, st, "twiddles", prism::launch_twiddles(w.twH, n / 2, st));
  LAUNCH(p, st, "twiddles", prism::launch_twiddles2(w.tw2, n, st));
  LAUNCH(p, st, "prop_lut", prism::launch_prop_lut(w.prop, n, g.ref->H, w.thick, g.ref->lam, g.ref->dq, st));
  // per member: transmissions and beam list; per wave: its member
  struct Seg {
    int item, first_beam, nb, H;
    const float2* trans;
    const int32_t* mn;
  };
  std::vector<Seg> waves_of;  // one segment per member, in wave order
  size_t toff = 0, moff = 0;
  for (int i : g.items) {
    const prism_build_item& it = items[i];
    const std::vector<int32_t>& mn = it.plan->beams.at({it.f, dbits(it.alpha_max_mrad)});
    float2* tr = w.trans + toff;
    LAUNCH(p, st, "transmission",
           prism::launch_transmission(it.plan->phase, tr, (size_t)it.plan->H * n * n,
                                      1.0f / (float)n, st));
    HIP_TRY(hipMemcpyAsync(w.mn + moff, mn.data(), mn.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy beam list");
    waves_of.push_back(Seg{i, 0, (int)(mn.size() / 2), it.plan->H, tr, w.mn + moff});
    toff += (size_t)it.plan->H * n * n;
    moff += mn.size();
  }
  const size_t splane = (size_t)(n / 2) * (n / 2), wave = (size_t)n * (n / 2);
  // walk the waves chunk by chunk (a member may span chunks)
  size_t seg = 0;
  int seg_b = 0;  // next beam of waves_of[seg]
  while (seg < waves_of.size()) {
    struct Part {
      const Seg* s;
      int b0, nb, w0;
    };
    std::vector<Part> parts;
    std::vector<uint64_t> tab;
    int used = 0;
    while (used < chunk && seg < waves_of.size()) {
      const Seg& sg = waves_of[seg];
      const int take = std::min(chunk - used, sg.nb - seg_b);
      parts.push_back(Part{&sg, seg_b, take, used});
      for (int k = 0; k < take; ++k) tab.push_back((uint64_t)(uintptr_t)sg.trans);
      used += take;
      seg_b += take;
      if (seg_b == sg.nb) {
        ++seg;
        seg_b = 0;
      }
    }
    const std::vector<uint64_t>& kept = *lead->batch_tables.insert(tab).first;
    HIP_TRY(hipMemcpyAsync(w.wtab, kept.data(), kept.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, st),
            "copy wave table");
    for (const Part& pt : parts) {
      const prism_build_item& it = items[pt.s->item];
      LAUNCH(p, st, "beam_init",
             prism::launch_beam_init(w.state + (size_t)pt.w0 * wave, pt.s->mn, pt.b0, pt.nb, n,
                                     it.f, w.twN, st));
    }
    // parts are in decreasing slice count: the first `active` waves still run
    const int hmax = parts.front().s->H;
    for (int s = 0; s < hmax; ++s) {
      int active = 0;
      for (const Part& pt : parts)
        if (pt.s->H > s) active = pt.w0 + pt.nb;
      LAUNCH(p, st, "row_pass",
             prism::launch_row_pass(w.state, active, n, nullptr, w.twN, w.tw2, p->tune, st,
                                    w.wtab, (size_t)s * n * n));
      LAUNCH(p, st, "col_pass",
             prism::launch_col_pass(w.state, active, n, w.prop + (size_t)s * n, w.twN, w.tw2,
                                    p->tune, st));
    }
    for (const Part& pt : parts) {
      const prism_build_item& it = items[pt.s->item];
      float2* S = static_cast<float2*>(it.smatrix_dev) + (size_t)pt.b0 * splane;
      LAUNCH(p, st, "extract",
             prism::launch_extract(w.state + (size_t)pt.w0 * wave, pt.nb, n, S, w.twH, st));
    }
  }
  return PRISM_OK;
}

}  // namespace

extern "C" {

int prism_build_batch_workspace_bytes(const prism_build_item* items, int count, size_t* pref,
                                      size_t* minimum) {
  if (!pref || !minimum || (count > 0 && !items)) return fail(PRISM_EINVAL, "null argument");
  if (count < 0) return fail(PRISM_EINVAL, "negative item count");
  std::vector<BatchGroup> groups;
  std::vector<int> alone;
  if (int r = batch_groups(items, count, &groups, &alone)) return r;
  *pref = *minimum = 0;
  for (const auto& g : groups) {
    BatchWs w;
    const int total = batch_total_waves(items, g);
    *pref = std::max(*pref, batch_layout(items, g, batch_pref_chunk(g.ref->n, total), &w, nullptr));
    *minimum = std::max(*minimum, batch_layout(items, g, 1, &w, nullptr));
  }
  for (int i : alone) {
    size_t p1, m1;
    if (int r = prism_build_workspace_bytes(items[i].plan, items[i].f, items[i].alpha_max_mrad, &p1,
                                            &m1))
      return r;
    *pref = std::max(*pref, p1);
    *minimum = std::max(*minimum, m1);
  }
  return PRISM_OK;
}

int prism_build_smatrix_batch(const prism_build_item* items, int count, void* ws, size_t ws_bytes,
                              void* stream) {
  if (count < 0) return fail(PRISM_EINVAL, "negative item count");
  if (count == 0) return PRISM_OK;
  if (!items) return fail(PRISM_EINVAL, "null argument");
  std::vector<BatchGroup> groups;
  std::vector<int> alone;
  if (int r = batch_groups(items, count, &groups, &alone)) return r;
  for (int i = 0; i < count; ++i) {
    if (!items[i].smatrix_dev) return fail(PRISM_EINVAL, "batch item " + std::to_string(i) + ": null S-matrix");
    const std::vector<int32_t>& mn =
        items[i].plan->beams.at({items[i].f, dbits(items[i].alpha_max_mrad)});
    if (items[i].smatrix_bytes < smatrix_need(items[i].plan, mn))
      return fail(PRISM_EINVAL, "batch item " + std::to_string(i) +
                                    ": S-matrix buffer smaller than prism_smatrix_bytes");
    if (!items[i].plan->phase)
      return fail(PRISM_ENOTREADY, "batch item " + std::to_string(i) + ": potential slices not set");
  }
  if (!ws) return fail(PRISM_EINVAL, "null device buffer");
  for (const auto& g : groups) {  // every group must fit before anything is enqueued
    BatchWs w;
    if (batch_layout(items, g, 1, &w, nullptr) > ws_bytes)
      return fail(PRISM_ENOSPACE, "workspace smaller than the batched build minimum");
  }
  for (int i : alone) {
    size_t p1, m1;
    if (int r = prism_build_workspace_bytes(items[i].plan, items[i].f, items[i].alpha_max_mrad, &p1,
                                            &m1))
      return r;
    if (m1 > ws_bytes) return fail(PRISM_ENOSPACE, "workspace smaller than the batched build minimum");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int i : alone) {
    const prism_build_item& it = items[i];
    if (int r = prism_build_smatrix(it.plan, it.f, it.alpha_max_mrad, it.smatrix_dev,
                                    it.smatrix_bytes, ws, ws_bytes, stream))
      return fail(r, "batch item " + std::to_string(i) + ": " + g_err);
  }
  for (const auto& g : groups)
    if (int r = batch_build_group(items, g, ws, ws_bytes, st)) return r;
  return PRISM_OK;
}

}  // extern "C"
