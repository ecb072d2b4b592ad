// PRISM probe step (Fig. 1d-f), second half: the window FFT, |Psi|^2 and
// the detector sums.
//
//   alpha_{m,n}(r0) = A(q) e^{-i chi(q)} e^{-2 pi i q.r0} / (W sqrt(B_A))
//   psi(r, r0)      = sum_{m,n} S_{m,n}(r) alpha_{m,n}(r0)      (Eq. PRISMfinal)
// inside the W x W window of Eq. RegionBounds (coefficients and window sum:
// probe16_kernels.hip), then |FFT_W psi|^2 / W^2 integrated per detector
// bin here, or stored whole (CBED).
#include <algorithm>

#include "fft_lds.hpp"
#include "fft_reg.hpp"
#include "kernels.hpp"

namespace prism {

namespace {

// Probe grouping of the window sum (shared with probe16_kernels.hip): probes
// per group for W >= 128, and the union tiles of 128 pixels.
constexpr int kCG128 = 64;
constexpr int kCTile = 128;

// ---------------------------------------------------------------------------
// W = 256 windows (too large for one workgroup's LDS): the 2D FFT runs as
// two four-step passes over the window buffer, 256 = 16 x 16.
//   rows : 16 lanes per row, lane j holds x = 16 a + j; DFT over a, twiddle
//          w_256^{jc}, LDS transpose, DFT over b -> row[c + 16 d], in place;
//   cols : tiles of 16 columns, lane (b, c) holds y = 16 a + b of column c;
//          the same steps along y, then I = |Psi|^2 / W^2 at full-grid
//          frequency f k_w is summed per detector bin (FP64) into one partial
//          per (probe, tile).
constexpr int kW4 = 256, kR4 = 16;

__device__ __forceinline__ void load_tw16(float2* twl, const float2* __restrict__ twW, int tid) {
  // twl[m][j] = w_256^{j m}
  twl[tid] = twW[((tid & 15) * (tid >> 4)) & (kW4 - 1)];
}

__global__ __launch_bounds__(256) void k_window_rows256(float2* __restrict__ window,
                                                        const float2* __restrict__ twW) {
  constexpr int R = kR4, LS = R + 1;
  __shared__ float2 twl[R * R];
  __shared__ float2 lds[R * R * LS];
  const int tid = threadIdx.x, j = tid % R, rr = tid / R;
  load_tw16(twl, twW, tid);
  __syncthreads();
  float2* row = window + ((size_t)blockIdx.x * R + rr) * kW4;
  float2* L = lds + rr * R * LS;
  float2 v[R];
#pragma unroll
  for (int a = 0; a < R; ++a) v[a] = row[R * a + j];
  dft_reg<R, false>(v);
#pragma unroll
  for (int c = 0; c < R; ++c) L[c * LS + j] = c ? cmul(v[c], twl[c * R + j]) : v[c];
  __syncthreads();
#pragma unroll
  for (int b = 0; b < R; ++b) v[b] = L[j * LS + b];
  dft_reg<R, false>(v);
#pragma unroll
  for (int d = 0; d < R; ++d) row[j + R * d] = v[d];
}

template <bool CBED, int NB>
__global__ __launch_bounds__(256) void k_window_cols256_detect(const float2* __restrict__ window,
                                                               const float2* __restrict__ twW,
                                                               int f, DetBins bins,
                                                               double* __restrict__ partial,
                                                               float* __restrict__ cbed,
                                                               OutAcc oa) {
  constexpr int R = kR4, LS = R + 1, TC = 16, TILES = kW4 / TC;
  constexpr int CS = R * LS + 1;  // column stride: 16 columns on distinct banks
  __shared__ float2 twl[R * R];
  __shared__ float2 lds[TC * CS];
  __shared__ double red[NB][4];
  const int tid = threadIdx.x, c = tid % TC, b = tid / TC;
  load_tw16(twl, twW, tid);
  __syncthreads();
  const size_t p = blockIdx.x / TILES;
  const int tile = blockIdx.x % TILES, col = tile * TC + c;
  const float2* src = window + p * kW4 * kW4 + col;
  float2* L = lds + c * CS;
  float2 v[R];
#pragma unroll
  for (int a = 0; a < R; ++a) v[a] = src[(size_t)(R * a + b) * kW4];
  dft_reg<R, false>(v);
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) L[k1 * LS + b] = k1 ? cmul(v[k1], twl[k1 * R + b]) : v[k1];
  __syncthreads();
#pragma unroll
  for (int bb = 0; bb < R; ++bb) v[bb] = L[b * LS + bb];
  dft_reg<R, false>(v);  // lane (k1 = b, c): ky index b + R k2
  const double inv_w2 = 1.0 / ((double)kW4 * (double)kW4);
  if constexpr (CBED) {
    float* dst = cbed + p * kW4 * kW4 + col;
#pragma unroll
    for (int k2 = 0; k2 < R; ++k2)
      put_out(dst + (size_t)(b + R * k2) * kW4,
              ((double)v[k2].x * v[k2].x + (double)v[k2].y * v[k2].y) * inv_w2, oa);
    return;
  }
  const long long kx = col < kW4 / 2 ? col : col - kW4;
  double acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = 0.0;
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) {
    const int kyi = b + R * k2;
    const long long ky = kyi < kW4 / 2 ? kyi : kyi - kW4;
    const long long kk = (long long)f * f * (kx * kx + ky * ky);
    const double I = ((double)v[k2].x * v[k2].x + (double)v[k2].y * v[k2].y) * inv_w2;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < bins.n && kk >= bins.lo[q] && kk < bins.hi[q]) acc[q] += I;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q < bins.n) {  // uniform
      const double sum = wave_sum(acc[q]);
      if ((tid & 63) == 0) red[q][tid >> 6] = sum;
    }
  }
  __syncthreads();
  if (tid < bins.n)
    partial[((size_t)p * TILES + tile) * bins.n + tid] =
        red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

// ---------------------------------------------------------------------------
// W = 144 and 192 (more than one workgroup's LDS, not a square of a register
// DFT length): the same two passes over the window buffer with the LDS
// Stockham transforms: rows (kBigRows per workgroup) in place, then tiles of
// 16 columns with |Psi|^2 / W^2 and per-element binning (or CBED) as for
// W = 256.
constexpr int kBigRows = 8, kBigTC = 16, kBigNT = 256;

template <int W>
__global__ __launch_bounds__(kBigNT) void k_window_rows_lds(float2* __restrict__ window,
                                                            const float2* __restrict__ twW) {
  using B = RowBatch<W, kBigRows>;
  __shared__ float2 lds[lds_padded(W * kBigRows)];
  __shared__ float2 tw[W];
  const int tid = threadIdx.x;
  load_twiddles<W, kBigNT>(tw, twW, tid);
  float2* rows = window + (size_t)blockIdx.x * kBigRows * W;
  for (int e = tid; e < kBigRows * W; e += kBigNT) lds[lpad(e)] = rows[e];
  __syncthreads();
  fft_lds<B, kBigNT, false>(lds, tw, tid);
  for (int e = tid; e < kBigRows * W; e += kBigNT) rows[e] = lds[lpad(e)];
}

template <int W, bool CBED, int NB>
__global__ __launch_bounds__(kBigNT) void k_window_cols_lds(const float2* __restrict__ window,
                                                            const float2* __restrict__ twW, int f,
                                                            DetBins bins,
                                                            double* __restrict__ partial,
                                                            float* __restrict__ cbed, OutAcc oa) {
  constexpr int TILES = W / kBigTC;
  using B = Batch<W, kBigTC, kBigTC, 0, 1, kBigTC, true>;  // [y][c], column c is sequence c
  __shared__ float2 lds[lds_padded(W * kBigTC)];
  __shared__ float2 tw[W];
  __shared__ double red[CBED ? 1 : NB][kBigNT / 64];
  const int tid = threadIdx.x;
  load_twiddles<W, kBigNT>(tw, twW, tid);
  const size_t p = blockIdx.x / TILES;
  const int tile = blockIdx.x % TILES;
  const float2* src = window + p * W * W + tile * kBigTC;
  for (int e = tid; e < W * kBigTC; e += kBigNT) lds[lpad(e)] = src[(e / kBigTC) * W + e % kBigTC];
  __syncthreads();
  fft_lds<B, kBigNT, false>(lds, tw, tid);
  const double inv_w2 = 1.0 / ((double)W * (double)W);
  if constexpr (CBED) {
    float* dst = cbed + p * W * W + tile * kBigTC;
    for (int e = tid; e < W * kBigTC; e += kBigNT) {
      const float2 z = lds[lpad(e)];
      put_out(dst + (e / kBigTC) * W + e % kBigTC, ((double)z.x * z.x + (double)z.y * z.y) * inv_w2,
              oa);
    }
    return;
  }
  double acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = 0.0;
  for (int e = tid; e < W * kBigTC; e += kBigNT) {
    const int kyi = e / kBigTC, col = tile * kBigTC + e % kBigTC;
    const long long kx = col < W / 2 ? col : col - W, ky = kyi < W / 2 ? kyi : kyi - W;
    const long long kk = (long long)f * f * (kx * kx + ky * ky);
    const float2 z = lds[lpad(e)];
    const double I = ((double)z.x * z.x + (double)z.y * z.y) * inv_w2;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q < bins.n && kk >= bins.lo[q] && kk < bins.hi[q]) acc[q] += I;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q < bins.n) {  // uniform
      const double sum = wave_sum(acc[q]);
      if ((tid & 63) == 0) red[q][tid >> 6] = sum;
    }
  }
  __syncthreads();
  if (tid < bins.n) {
    double sm = 0.0;
    for (int w = 0; w < kBigNT / 64; ++w) sm += red[tid][w];
    partial[((size_t)p * TILES + tile) * bins.n + tid] = sm;
  }
}

// ---------------------------------------------------------------------------
#ifndef PRISM_WD_GRID
#define PRISM_WD_GRID 1048576  // window kernel: most workgroups (each then walks probes)
#endif
#ifndef PRISM_WD128_NT
#define PRISM_WD128_NT 1024  // threads per W = 128 window workgroup
#endif
constexpr int kWdChunks = 16;  // bin-list chunks whose pixel indices load together

// Threads per window workgroup: W^2 / 16 rounded up to whole waves.
__host__ __device__ constexpr int wd_nt(int w) {
  return w == 128 ? PRISM_WD128_NT : ((w * w / 16) < 64 ? 64 : (w * w / 16 + 63) / 64 * 64);
}

// 2D FFT of each W x W window in LDS, then either I(kw) = |Psi(kw)|^2 / W^2
// summed over each bin's pixel list in FP64 (the lists encode the angle test
// at full-grid frequency f kw), or (CBED) I written out in full. Workgroups
// walk windows p = blockIdx.x, + gridDim.x, ... (one window each unless
// there are more than PRISM_WD_GRID); window p belongs to the segment whose
// range holds it (its own outputs and, for the sums, its own pixel lists).
//
// Bin sums: the lists are cut into chunks of kWdListChunk = 64 entries (one
// per lane, kNoPix padding at the end of each bin); chunk k belongs to the
// bin j with off[j] <= k < off[j + 1]. Wave w takes the contiguous chunks
// [K w / NW, K (w + 1) / NW) of the K in all, so it meets only a few bins:
// each lane sums its entry of the wave's chunks of a bin in order, one wave
// sum per bin met goes to red[j][w] (zero for the bins a wave does not
// meet), and the bin total adds red[j][0 .. NW) in order. The pixel indices
// of kWdChunks chunks are loaded together, so the load latency is paid once
// per group of chunks.
template <int W, bool CBED>
__global__ __launch_bounds__(wd_nt(W)) void k_window_detect(const float2* __restrict__ window,
                                                            const float2* __restrict__ twW,
                                                            const WindowSegs segs) {
  constexpr int NT = wd_nt(W);
  constexpr int NW = NT / 64;
  // first row stage, applied from registers: radix 8 where W allows, else
  // 4, 2 or 3 (W = 12, 36: 4; W = 18: 2)
  constexpr int R0 = W % 8 == 0 ? 8 : (W % 4 == 0 ? 4 : (W % 2 == 0 ? 2 : 3));
  using Rows = RowBatch<W, W>;
  using Cols = Batch<W, W, W, 0, 1, W, true>;
  using S8 = StageShape<Rows, R0, NT>;
  __shared__ float2 lds[lds_padded(W * W)];
  __shared__ float2 tw[W];
  __shared__ double red[CBED ? 1 : kMaxDet][NW];
  const int tid = threadIdx.x;
  load_twiddles<W, NT>(tw, twW, tid);
  const double inv_w2 = 1.0 / ((double)W * (double)W);
#pragma unroll 1
  for (int p = blockIdx.x; p < segs.total; p += gridDim.x) {
    int k = 0;  // segment of window p (uniform)
    while (k + 1 < segs.n && p >= segs.s[k + 1].begin) ++k;
    const WindowSeg& sg = segs.s[k];
    const int q = p - sg.begin;  // probe within the segment
    float2 v[S8::PER][R0];
    {
      const float2* src = window + (size_t)p * W * W;
#pragma unroll
      for (int c = 0; c < S8::PER; ++c) {
        const int b = tid + c * NT;
        if (!S8::GUARD || b < S8::TOT) {
          int row, j;
          stage_coords<Rows, S8::NB>(b, row, j);
#pragma unroll
          for (int r = 0; r < R0; ++r) v[c][r] = src[row * W + j + r * (W / R0)];
        }
      }
    }
    stage_out<Rows, R0, 1, NT, false>(lds, tid, v);
    __syncthreads();
    fft_from<Rows, NT, false, R0>(lds, tw, tid);
    fft_lds<Cols, NT, false>(lds, tw, tid);
    if constexpr (CBED) {
      float* dst = sg.cbed + (size_t)q * W * W;
      for (int e = tid; e < W * W; e += NT) {
        const float2 z = lds[lpad(e)];
        put_out(dst + e, ((double)z.x * z.x + (double)z.y * z.y) * inv_w2, sg.oa);
      }
    } else {
      const uint16_t* __restrict__ pix = sg.pix;
      const BinLists* __restrict__ lists = sg.lists;  // uniform: scalar loads
      const int nb = lists->n;
      const int* off = lists->off;
      const int K = off[nb];  // chunks of kWdListChunk entries
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
      for (int i = tid; i < nb * NW; i += NT) red[i / NW][i % NW] = 0.0;
      __syncthreads();
      const int c0 = (int)((long long)K * wv / NW), c1 = (int)((long long)K * (wv + 1) / NW);
      int j = 0;  // bin of the current chunk (uniform in the wave)
      while (j < nb && c0 >= off[j + 1]) ++j;
      double acc = 0.0;
      for (int k0 = c0; k0 < c1; k0 += kWdChunks) {
        int px[kWdChunks];
#pragma unroll
        for (int c = 0; c < kWdChunks; ++c)
          px[c] = k0 + c < c1 ? (int)pix[(size_t)(k0 + c) * kWdListChunk + lane] : (int)kNoPix;
#pragma unroll
        for (int c = 0; c < kWdChunks; ++c) {
          const int kk = k0 + c;
          if (kk < c1) {
            if (kk >= off[j + 1]) {  // bin j ends: its wave sum, then the bin of chunk kk
              const double sm = wave_sum(acc);
              if (lane == 0) red[j][wv] = sm;
              acc = 0.0;
              do ++j;
              while (kk >= off[j + 1]);
            }
            const bool ok = px[c] != (int)kNoPix;
            const float2 z = lds[lpad(ok ? px[c] : 0)];
            const double I = (double)z.x * z.x + (double)z.y * z.y;
            acc += ok ? I : 0.0;
          }
        }
      }
      if (c1 > c0) {
        const double sm = wave_sum(acc);
        if (lane == 0) red[j][wv] = sm;
      }
      __syncthreads();
      if (tid < nb) {
        double sm = 0.0;
        for (int w = 0; w < NW; ++w) sm += red[tid][w];
        put_out(sg.out + (size_t)q * nb + tid, sm * inv_w2, sg.oa);
      }
    }
    __syncthreads();  // LDS free for the next window
  }
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int contract_group(int w) { return w >= 128 ? kCG128 : (w >= 64 ? 32 : 16); }

int contract_tile_slots(int w, int window_tile_div) {
  const int own = (w * w + kCTile - 1) / kCTile;  // tiles of one window
  return std::max(1, own / std::max(1, window_tile_div));
}

int window_big_tiles(int w) { return w / 16; }

// Accumulator slots of the per-element binning kernels for n bins: the
// smallest of 4, 8, 16 and kMaxDet that holds them (the kernels test each
// element against every slot below n, so fewer slots mean less work per
// element; the sums are the same).
static int bin_slots(int n) { return n <= 4 ? 4 : (n <= 8 ? 8 : (n <= 16 ? 16 : kMaxDet)); }

hipError_t launch_window_big(float2* window, int np, int w, const float2* twW, int f,
                             const DetBins& bins, double* partial, float* cbed, OutAcc acc,
                             hipStream_t st) {
  const bool want_cbed = cbed != nullptr;
  if (w == kW4) {
    hipLaunchKernelGGL(k_window_rows256, dim3((unsigned)((size_t)np * kW4 / kR4)), dim3(256), 0,
                       st, window, twW);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((size_t)np * window_big_tiles(w)));
    if (want_cbed) {
      hipLaunchKernelGGL((k_window_cols256_detect<true, 1>), grid, dim3(256), 0, st, window, twW,
                         f, bins, (double*)nullptr, cbed, acc);
      return hipGetLastError();
    }
#define C256(NBB)                                                                          \
  hipLaunchKernelGGL((k_window_cols256_detect<false, NBB>), grid, dim3(256), 0, st, window, \
                     twW, f, bins, partial, (float*)nullptr, OutAcc{})
    switch (bin_slots(bins.n)) {
      case 4: C256(4); break;
      case 8: C256(8); break;
      case 16: C256(16); break;
      default: C256(kMaxDet); break;
    }
#undef C256
    return hipGetLastError();
  }
#define WCOLS(WW, NBB)                                                                     \
  hipLaunchKernelGGL((k_window_cols_lds<WW, false, NBB>), grid, dim3(kBigNT), 0, st, window, \
                     twW, f, bins, partial, (float*)nullptr, OutAcc{})
#define WBIG(WW)                                                                           \
  case WW: {                                                                               \
    hipLaunchKernelGGL(k_window_rows_lds<WW>, dim3((unsigned)((size_t)np * WW / kBigRows)), \
                       dim3(kBigNT), 0, st, window, twW);                                  \
    hipError_t e = hipGetLastError();                                                      \
    if (e != hipSuccess) return e;                                                         \
    const dim3 grid((unsigned)((size_t)np * (WW / kBigTC)));                               \
    if (want_cbed) {                                                                       \
      hipLaunchKernelGGL((k_window_cols_lds<WW, true, 1>), grid, dim3(kBigNT), 0, st,      \
                         window, twW, f, bins, (double*)nullptr, cbed, acc);               \
      break;                                                                               \
    }                                                                                      \
    switch (bin_slots(bins.n)) {                                                           \
      case 4: WCOLS(WW, 4); break;                                                         \
      case 8: WCOLS(WW, 8); break;                                                         \
      case 16: WCOLS(WW, 16); break;                                                       \
      default: WCOLS(WW, kMaxDet); break;                                                  \
    }                                                                                      \
    break;                                                                                 \
  }
  switch (w) {
    WBIG(144)
    WBIG(192)
    default:
      return hipErrorInvalidValue;
  }
#undef WBIG
#undef WCOLS
  return hipGetLastError();
}

// Workgroups for the window kernels: one per probe up to PRISM_WD_GRID, then
// each walks several probes.
static unsigned window_grid(int np) { return (unsigned)std::min(np, PRISM_WD_GRID); }

hipError_t launch_window_detect(const float2* window, const WindowSegs& segs, int w,
                                const float2* twW, hipStream_t st) {
  if (segs.total <= 0) return hipSuccess;
  if (segs.n < 1 || segs.n > kMaxSeg) return hipErrorInvalidValue;
#define WD(WW)                                                                          \
  case WW:                                                                              \
    hipLaunchKernelGGL((k_window_detect<WW, false>), dim3(window_grid(segs.total)),     \
                       dim3(wd_nt(WW)), 0, st, window, twW, segs);                      \
    break;
  switch (w) {
    WD(8)
    WD(16)
    WD(32)
    WD(64)
    WD(128)
    WD(24)
    WD(48)
    WD(72)
    WD(96)
    WD(12)
    WD(18)
    WD(36)
    default:
      return hipErrorInvalidValue;
  }
#undef WD
  return hipGetLastError();
}

hipError_t launch_window_cbed(const float2* window, const WindowSegs& segs, int w,
                              const float2* twW, hipStream_t st) {
  if (segs.total <= 0) return hipSuccess;
  if (segs.n < 1 || segs.n > kMaxSeg) return hipErrorInvalidValue;
#define WC(WW)                                                                          \
  case WW:                                                                              \
    hipLaunchKernelGGL((k_window_detect<WW, true>), dim3(window_grid(segs.total)),      \
                       dim3(wd_nt(WW)), 0, st, window, twW, segs);                      \
    break;
  switch (w) {
    WC(8)
    WC(16)
    WC(32)
    WC(64)
    WC(128)
    WC(24)
    WC(48)
    WC(72)
    WC(96)
    WC(12)
    WC(18)
    WC(36)
    default:
      return hipErrorInvalidValue;
  }
#undef WC
  return hipGetLastError();
}

}  // namespace prism
