// Launch interface between the host plan (plan.cpp) and the HIP kernels.
//
// Wave state layout used by both the S-matrix build and multislice STEM:
// after the x-transform of a slice step, a wave is held as
//     X(y, kx) = sum_x psi(x, y) exp(-2 pi i kx x / n)
// for the n/2 columns |kx| < n/4 that survive the half-band aperture
// (compact column jj in [0, n/2) holds kx = jj for jj < n/4, else jj - n/2,
// i.e. n/2-point fftfreq order). Layout: c64 [wave][y][n/2]. Columns with
// |kx| >= n/4 are identically zero after every propagator step, so they are
// never stored; this halves the HBM traffic of each pass.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace prism {

constexpr int kMaxDet = 32;

// Detector bins as half-open integer ranges of full-grid |k|^2:
// bin j holds lo[j] <= kx^2 + ky^2 < hi[j]. Decided on the host in FP64
// from theta = (lambda dq) sqrt(k^2) so that the kernels only compare ints.
struct DetBins {
  int n;
  int lo[kMaxDet];
  int hi[kMaxDet];
};

// How a kernel stores a result v into an output element: overwrite (on = 0)
// or add w * v to what is there (on = 1; the average over frozen-phonon
// configurations is a sum of calls with w = 1/K).
struct OutAcc {
  int on;
  double w;
};
__host__ __device__ inline void put_out(double* o, double v, OutAcc a) {
  *o = a.on ? *o + a.w * v : v;
}
__host__ __device__ inline void put_out(float* o, double v, OutAcc a) {
  *o = a.on ? (float)((double)*o + a.w * v) : (float)v;
}

// Per-probe optics for the GPU-side FP64 phase computations.
struct ProbeOptics {
  double lam;      // wavelength (A)
  double dq;       // 1 / cell (1/A)
  double C1, C3;   // aberrations (A)
  double cell;     // cell side (A)
  double ktx, kty; // tilt as a full-grid frequency offset: chi is taken at k - k_t
  double sx, sy;   // entrance offset h tan(theta_t) (A): positions enter as r0 - s
  double norm;     // incident-wave normalisation factor
};

// Launch shapes that do not change any result (work distribution only):
// the four-step slice passes' iteration caps and smallest grids, and the
// window sum's workgroups per probe group (union tiles of one window /
// window_tile_div). Set per plan (prism_set_tuning); defaults below.
struct LaunchTuning {
  int row_iters = 16;      // most row groups per workgroup (power of two)
  int row_min_wg = 512;    // fewest workgroups per row-pass launch
  int col_iters = 8;       // most column tiles per workgroup (power of two)
  int col_min_wg = 256;    // fewest workgroups per column-pass launch
  int window_tile_div = 4;
};

hipError_t launch_twiddles(float2* tw, int L, hipStream_t st);
hipError_t launch_transmission(const float* phase, float2* trans, size_t count, float scale,
                               hipStream_t st);
// lut[p][i] = exp(-i pi lambda t_p (k dq)^2) for full-grid index i (k in fftfreq order).
hipError_t launch_prop_lut(float2* lut, int n, int H, const double* thick_dev, double lam,
                           double dq, hipStream_t st);

hipError_t launch_beam_init(float2* state, const int32_t* beams_mn, int b0, int nb, int n, int f,
                            const float2* twN, hipStream_t st);
// aper[ky + n/2] = (kx_lo, kx_hi): the aperture's full-grid pixels of row ky
// (empty when kx_lo > kx_hi), decided on the host.
hipError_t launch_probe_init(float2* state, const double* probe_xy, int p0, int np, int n,
                             const ProbeOptics& po, const int2* aper, const float2* twN,
                             hipStream_t st);
// Four-step slice passes (n = R^2): R, or 0 where the Stockham kernels run.
int four_step_radix(int n);
// tw2[m][j] = exp(-2 pi i j m / n), j, m < R (n entries; nothing for R = 0).
hipError_t launch_twiddles2(float2* tw2, int n, hipStream_t st);
// wtrans != nullptr: wave w multiplies by wtrans[w] + soff instead of trans_p
// (device table of per-wave transmission bases: waves of several specimens
// in one launch).
hipError_t launch_row_pass(float2* state, int nwaves, int n, const float2* trans_p,
                           const float2* twN, const float2* tw2, const LaunchTuning& tune,
                           hipStream_t st, const float2* const* wtrans = nullptr,
                           size_t soff = 0);
hipError_t launch_col_pass(float2* state, int nwaves, int n, const float2* prop_p,
                           const float2* twN, const float2* tw2, const LaunchTuning& tune,
                           hipStream_t st);
// Last slice of multislice STEM: FFT_y, propagator, band limit, |Psi|^2/n^2
// and per-column-tile detector partial sums (double [wave][tiles][n_det]).
hipError_t launch_col_detect(const float2* state, int nwaves, int n, const float2* prop_p,
                             const float2* twN, const DetBins& bins, double* partial,
                             hipStream_t st);
int col_tiles(int n);
hipError_t launch_reduce_partials(const double* partial, int nwaves, int tiles, int n_det,
                                  double* out, OutAcc acc, hipStream_t st);
hipError_t launch_extract(const float2* state, int nwaves, int n, float2* smatrix,
                          const float2* twH, hipStream_t st);

// PRISM probe step.
struct ActiveBeam {
  int plane;  // index of the beam's plane in the S-matrix
  int m, n;   // plane-wave indices
};

// Probes per group of the packed window sum (they share one union window):
// the default for window side w.
int contract_group(int w);
// Workgroups per probe group along the union tiles (each loops over tiles).
int contract_tile_slots(int w, int window_tile_div);

// Low-precision probe step (BF16 or FP16 operands, FP32 accumulation).
// Operand forms of the packed window sum: 16-bit (BF16, FP16; one 32-bit
// word per complex value, 32 beams per K block) or FP32 (two words per
// value, 16 beams per K block). A K block is 128 bytes of a pixel row.
enum class Prec { kBF16 = 1, kFP16 = 2, kF32 = 3 };
constexpr int kC16KB = 32;  // 32-bit words per K block row
__host__ __device__ constexpr int prec_block_beams(Prec p) { return p == Prec::kF32 ? 16 : 32; }
__host__ __device__ constexpr int prec_words(Prec p) { return p == Prec::kF32 ? 2 : 1; }
// Beam rows of the packed S-matrix are padded to a whole pair of K blocks.
__host__ __device__ constexpr int prec_beam_pad(Prec p) { return 2 * prec_block_beams(p); }
// scale[a] = 2^-e with e the smallest integer such that every |Re|, |Im| of
// active beam a's plane is < 2^e (1 for an all-zero plane); partial holds
// n_act * kScaleSplit floats of per-block maxima (ns >= 64).
constexpr int kScaleSplit = 32;
hipError_t launch_s16_scale(const float2* smatrix, const ActiveBeam* act, int n_act, int ns,
                            float* partial, float* scale, hipStream_t st);
// s16 [ns*ns][n_actp][2] 16-bit: (Re, Im) of scale[a] * S_a(pixel); zero for a >= n_act.
hipError_t launch_s16_pack(const float2* smatrix, const ActiveBeam* act, int n_act, int n_actp,
                           int ns, const float* scale, void* s16, Prec prec, hipStream_t st);
// a16: per probe group and 32-beam block, the real-ified A' block [2G][64] in
// 16 bits of alpha'' = exp(i phase) / scale[a]; also the window origins.
hipError_t launch_alpha16(const double* probe_xy, int p0, int np, const ActiveBeam* act,
                          int n_act, int n_actp, int f, int ns, int w, const ProbeOptics& po,
                          const float* scale, int group, void* a16, int2* origin, Prec prec,
                          hipStream_t st);
// Segments of one window-sum launch: the probe groups of several requests
// (specimens, optics) that share the window side, operand form and group
// size. Segment k owns the launch's groups g_begin .. g_begin +
// ceil(np / G) (its probes' A blocks at a16, group-major) and writes the
// windows of its np probes from window on (contiguous, probe order).
constexpr int kMaxSeg = 16;
struct ContractSeg {
  const uint32_t* s16;  // packed S of its specimen: [ns^2][rowlen] words
  const uint32_t* a16;  // [groups][K blocks][2G][32 words]
  const int2* origin;   // [np] window origins
  float2* window;       // [np][w][w]
  int rowlen;           // 32-bit words per packed pixel row
  int ns;               // S-matrix side (n / 2)
  int np;               // probes
  int g_begin;          // first group of the launch's grid
  float out_scale;      // 1 / (W sqrt(B_A)) of its active beams
};
struct ContractSegs {
  int n;       // segments
  int groups;  // groups over all segments
  ContractSeg s[kMaxSeg];
};
hipError_t launch_contract16(const ContractSegs& segs, int w, int group, Prec prec,
                             int window_tile_div, hipStream_t st);
// Detector bins as lists of window pixels (v * W + u of the W x W window),
// cut into chunks of kWdListChunk entries: bin j owns the chunks
// off[j] .. off[j+1]), i.e. pix[off[j] 64 .. off[j+1] 64), its last chunk
// padded with kNoPix.
struct BinLists {
  int n;
  int off[kMaxDet + 1];
};
constexpr int kWdListChunk = 64;  // one entry per lane of a wave
constexpr uint16_t kNoPix = 0xFFFF;
// Windows larger than 128 (W = 144, 192, 256): window FFT in two passes over
// the window buffer (rows in place, then tiles of 16 columns fused with
// |Psi|^2 / W^2 and per-element bin sums) into partial[probe][tile][n_det],
// tiles = window_big_tiles(w), reduced with launch_reduce_partials; or,
// with cbed != nullptr, cbed[p][ky][kx] = |Psi|^2 / W^2 (float32, fftfreq
// order) stored or accumulated by acc. W = 256 runs four-step 16 x 16
// passes, W = 144 and 192 LDS Stockham passes.
__host__ __device__ constexpr bool window_big(int w) { return w > 128; }
int window_big_tiles(int w);
hipError_t launch_window_big(float2* window, int np, int w, const float2* twW, int f,
                             const DetBins& bins, double* partial, float* cbed, OutAcc acc,
                             hipStream_t st);
// Window sides: in one workgroup's LDS the powers of two 8..128 and the
// 3 * 2^k / 9 * 2^k sides 12, 18, 24, 36, 48, 72, 96; over HBM (two passes)
// 144, 192 and 256.
__host__ __device__ constexpr bool window_side_ok(int w) {
  return w == 8 || w == 16 || w == 32 || w == 64 || w == 128 || w == 12 || w == 18 ||
         w == 24 || w == 36 || w == 48 || w == 72 || w == 96 || w == 144 || w == 192 ||
         w == 256;
}
// Segments of one window launch (W <= 128): windows begin .. next begin
// (or total) of the window buffer belong to segment k, whose probe q =
// window - begin stores into out[q][n_det] (detector sums, pixel lists pix
// with the device copy lists of their offsets) or cbed[q][W][W].
struct WindowSeg {
  const uint16_t* pix;
  const BinLists* lists;
  double* out;
  float* cbed;
  OutAcc oa;
  int begin;
};
struct WindowSegs {
  int n;      // segments
  int total;  // windows
  WindowSeg s[kMaxSeg];
};
// Full CBED output: cbed[p][ky][kx] = |FFT_W window_p|^2 / W^2 (float32,
// window fftfreq order), W <= 128 (larger windows: launch_window_big).
hipError_t launch_window_cbed(const float2* window, const WindowSegs& segs, int w,
                              const float2* twW, hipStream_t st);
hipError_t launch_window_detect(const float2* window, const WindowSegs& segs, int w,
                                const float2* twW, hipStream_t st);

}  // namespace prism
