// PRISM probe step (Fig. 1d-f): coefficients, window sum, FFT, detectors.
//
//   alpha_{m,n}(r0) = A(q) e^{-i chi(q)} e^{-2 pi i q.r0} / (W sqrt(B_A))
//   psi(r, r0)      = sum_{m,n} S_{m,n}(r) alpha_{m,n}(r0)      (Eq. PRISMfinal)
// inside the W x W window of Eq. RegionBounds, then |FFT_W psi|^2 / W^2
// integrated per detector bin.
//
// The window sum is a complex GEMM when neighbouring probes share their
// windows: for a group of G probes the union of their windows U is one
// M = 2G (real/imag rows) x N = |U| pixels x K = 2 B_A product with
//   A'[2g  ][2b] =  Re a_gb, A'[2g  ][2b+1] = -Im a_gb,
//   A'[2g+1][2b] =  Im a_gb, A'[2g+1][2b+1] =  Re a_gb,
//   B'[2b][x] = Re S_b(x),   B'[2b+1][x]   = Im S_b(x),
// run on v_mfma_f32_16x16x4f32 with FP32 accumulation. Each output pixel
// of the union is kept for the probes whose own window contains it.
#include <algorithm>

#include "fft_lds.hpp"
#include "fft_reg.hpp"
#include "kernels.hpp"

namespace prism {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap_mod(long long v, int m) {
  long long r = v % m;
  return (int)(r < 0 ? r + m : r);
}

// One thread per (active beam, probe); alpha is stored beam-major
// [n_act][np] so that a probe group's coefficients for one beam are
// contiguous. Also writes each probe's window origin (first S pixel of the
// cut-out, periodic).
__global__ void k_alpha(const double* __restrict__ probe_xy, int p0, int np,
                        const ActiveBeam* __restrict__ act, int n_act, int f, int ns, int w,
                        ProbeOptics po, float2* __restrict__ alpha, int2* __restrict__ origin) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)np * n_act) return;
  const int a = (int)(i / np), p = (int)(i % np);
  const double x0 = probe_xy[2 * (size_t)(p0 + p)], y0 = probe_xy[2 * (size_t)(p0 + p) + 1];
  if (a == 0) {
    const double dxs = po.cell / (double)ns;
    const int cx = wrap_mod((long long)floor(x0 / dxs + 0.5), ns);
    const int cy = wrap_mod((long long)floor(y0 / dxs + 0.5), ns);
    origin[p] = make_int2(wrap_mod((long long)cx - w / 2, ns), wrap_mod((long long)cy - w / 2, ns));
  }
  const double kx = (double)act[a].m * f, ky = (double)act[a].n * f;
  const double dx = kx - po.ktx, dy = ky - po.kty;
  const double q2 = (dx * dx + dy * dy) * (po.dq * po.dq);
  double t = -(0.5 * po.lam * q2 * po.C1 + 0.25 * po.lam * po.lam * po.lam * q2 * q2 * po.C3) -
             (kx * (x0 - po.sx) + ky * (y0 - po.sy)) * po.dq;
  t -= floor(t);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  alpha[i] = make_float2((float)(c * po.norm), (float)(s * po.norm));
}

// Contraction tile shape (tuned on MI355X; overridable at build time).
#ifndef PRISM_CKB
#define PRISM_CKB 16   // beams per K block
#endif
#ifndef PRISM_CCT
#define PRISM_CCT 2    // 16-pixel MFMA column tiles per wave
#endif
#ifndef PRISM_CG128
#define PRISM_CG128 64 // probes per group for W >= 128
#endif
#ifndef PRISM_CTILES_PER_WG
#define PRISM_CTILES_PER_WG 4  // union tiles per workgroup for a single window
#endif
constexpr int kCNT = 256;                 // threads per contraction workgroup (4 waves)
constexpr int kCCT = PRISM_CCT;
constexpr int kCTile = 4 * 16 * kCCT;     // union pixels per workgroup
constexpr int kCKB = PRISM_CKB;

struct UnionGeom {
  int y0, x0;  // first S pixel of the union (periodic)
  int uy, ux;  // union extent
};

// Contract one 128-pixel tile of the union for all G probes of the group.
// only < 0: write every probe whose window holds a pixel; only >= 0: write
// that probe alone (scattered groups). The K loop is double buffered: the
// next 16-beam block of alpha and S is fetched into registers while the
// MFMAs consume the current block from LDS.
template <int G>
struct ContractLds {
  static constexpr int AROW = 2 * G + 16;        // A'[k'][m'] row pitch (floats)
  static constexpr int BROW = kCTile + 16;       // B'[k'][n] row pitch (floats)
  static constexpr int ABUF = 2 * kCKB * AROW;   // floats per A' buffer
  static constexpr int BBUF = 2 * kCKB * BROW;   // floats per B' buffer
  static constexpr int FLOATS = 2 * (ABUF + BBUF);
};

template <int G>
__device__ __forceinline__ void contract_tile(const float2* __restrict__ S,
                                              const ActiveBeam* __restrict__ act, int n_act,
                                              const float2* __restrict__ alpha, int np,
                                              int p_base, int gcount, int ns, int w,
                                              const UnionGeom& U,
                                              int tile, const int* offx, const int* offy, int only,
                                              float* __restrict__ smem,
                                              float2* __restrict__ window) {
  using CL = ContractLds<G>;
  constexpr int RT = G / 8;                 // 16-row MFMA tiles covering 2G real rows
  constexpr int NA = G * kCKB / kCNT;       // alpha values staged per thread
  constexpr int NSV = kCKB * kCTile / kCNT; // S values staged per thread
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int npix = U.uy * U.ux;

  // pixel this thread stages for the S block (fixed across K blocks)
  const int n_ld = tid & (kCTile - 1);
  // beam row of the S block this wave stages: uniform per wave, so the
  // plane lookups below become scalar loads
  const int bl0 = __builtin_amdgcn_readfirstlane(tid / kCTile);
  const int up_ld = tile * kCTile + n_ld;
  long long soff = -1;
  if (up_ld < npix) {
    const int a = up_ld / U.ux, b = up_ld - a * U.ux;
    soff = (long long)((U.y0 + a) % ns) * ns + ((U.x0 + b) % ns);
  }
  const size_t plane = (size_t)ns * ns;

  // Two register sets: the block after next is in flight while a block is
  // computed. Loads are issued unconditionally from clamped (in-bounds)
  // indices and out-of-range entries are zeroed when staged, so the number
  // of loads in flight is the same on every path and each wait covers only
  // the older set.
  float2 ra[2][NA], rs[2][NSV];
  const long long soff_c = soff < 0 ? 0 : soff;
  auto fetch = [&](int set, int kb) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * kCNT;
      const int g = e % G, bl = e / G;
      const int b = min(kb + bl, n_act - 1), pidx = min(p_base + g, np - 1);
      ra[set][i] = alpha[(size_t)b * np + pidx];
    }
#pragma unroll
    for (int i = 0; i < NSV; ++i) {
      const int bl = bl0 + i * (kCNT / kCTile);
      rs[set][i] = S[(size_t)act[min(kb + bl, n_act - 1)].plane * plane + soff_c];
    }
  };
  // Stage one K block in the real MFMA operand layout:
  //   A'[2b][2g] = Re a, A'[2b+1][2g] = -Im a, A'[2b][2g+1] = Im a, A'[2b+1][2g+1] = Re a
  //   B'[2b][n]  = Re S, B'[2b+1][n] = Im S
  auto stash = [&](int set, int kb) {  // register set s goes to LDS buffer s
    float* A = smem + set * CL::ABUF;
    float* Bm = smem + 2 * CL::ABUF + set * CL::BBUF;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * kCNT;
      const int g = e % G, bl = e / G;
      const bool ok = g < gcount && kb + bl < n_act;
      const float2 a = ok ? ra[set][i] : make_float2(0.f, 0.f);
      *reinterpret_cast<float2*>(A + (2 * bl) * CL::AROW + 2 * g) = a;
      *reinterpret_cast<float2*>(A + (2 * bl + 1) * CL::AROW + 2 * g) = make_float2(-a.y, a.x);
    }
#pragma unroll
    for (int i = 0; i < NSV; ++i) {
      const int bl = bl0 + i * (kCNT / kCTile);
      const bool ok = soff >= 0 && kb + bl < n_act;
      Bm[(2 * bl) * CL::BROW + n_ld] = ok ? rs[set][i].x : 0.f;
      Bm[(2 * bl + 1) * CL::BROW + n_ld] = ok ? rs[set][i].y : 0.f;
    }
  };

  floatx4 acc[RT][kCCT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < kCCT; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int krow = lane >> 4, mcol = lane & 15;
  auto compute = [&](int buf) {
    const float* A = smem + buf * CL::ABUF + krow * CL::AROW + mcol;
    const float* Bm =
        smem + 2 * CL::ABUF + buf * CL::BBUF + krow * CL::BROW + 16 * kCCT * wv + mcol;
    // operands of K step ks+1 are read while the MFMAs of step ks run
    float av[2][RT], bv[2][kCCT];
#pragma unroll
    for (int r = 0; r < RT; ++r) av[0][r] = A[16 * r];
#pragma unroll
    for (int c = 0; c < kCCT; ++c) bv[0][c] = Bm[16 * c];
#pragma unroll
    for (int ks = 0; ks < kCKB / 2; ++ks) {
      const int cur = ks & 1, nxt = cur ^ 1;
      if (ks + 1 < kCKB / 2) {
#pragma unroll
        for (int r = 0; r < RT; ++r) av[nxt][r] = A[4 * (ks + 1) * CL::AROW + 16 * r];
#pragma unroll
        for (int c = 0; c < kCCT; ++c) bv[nxt][c] = Bm[4 * (ks + 1) * CL::BROW + 16 * c];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep those reads ahead of this step's MFMAs
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < kCCT; ++c)
          acc[r][c] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(av[cur][r], bv[cur][c], acc[r][c], 0, 0, 0);
    }
  };
  // K blocks alternate between register set / LDS buffer 0 and 1, in pairs;
  // an odd last block is paired with a zero-weight block.
  const int npair = (n_act + 2 * kCKB - 1) / (2 * kCKB);
  fetch(0, 0);
  fetch(1, kCKB);
  for (int pr = 0; pr < npair; ++pr) {
    const int kb = 2 * kCKB * pr;
    stash(0, kb);
    __syncthreads();
    fetch(0, kb + 2 * kCKB);
    compute(0);
    stash(1, kb + kCKB);
    __syncthreads();
    fetch(1, kb + 3 * kCKB);
    compute(1);
  }
  __syncthreads();  // LDS buffers free for a following tile

  // epilogue: lane holds rows 4*(lane/16)+i of each 16x16 tile, column lane%16
  const size_t w2 = (size_t)w * w;
#pragma unroll
  for (int c = 0; c < kCCT; ++c) {
    const int up = tile * kCTile + 16 * kCCT * wv + 16 * c + (lane & 15);
    if (up >= npix) continue;
    const int a = up / U.ux, b = up - a * U.ux;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int g = 8 * r + 2 * (lane >> 4) + h;
        if (g >= gcount || (only >= 0 && g != only)) continue;
        const int v = a - offy[g], u = b - offx[g];
        if (v < 0 || v >= w || u < 0 || u >= w) continue;
        window[(size_t)(p_base + g) * w2 + (size_t)v * w + u] =
            make_float2(acc[r][c][2 * h], acc[r][c][2 * h + 1]);
      }
    }
  }
}

template <int G>
__global__ __launch_bounds__(kCNT) __attribute__((amdgpu_waves_per_eu(2))) void k_contract(const float2* __restrict__ S,
                                                   const ActiveBeam* __restrict__ act, int n_act,
                                                   const float2* __restrict__ alpha,
                                                   const int2* __restrict__ origin, int np, int ns,
                                                   int w, float2* __restrict__ window) {
  __shared__ float smem[ContractLds<G>::FLOATS];  // two A' and two B' buffers
  __shared__ int offx[G], offy[G];
  __shared__ int ginfo[6];
  const int tid = threadIdx.x;
  const int p_base = blockIdx.y * G;
  const int gcount = min(G, np - p_base);
  if (tid < 64) {
    // group geometry in wave 0, one lane per probe (G <= 64): offsets of
    // each window from the first, their extent, and the union origin
    const int2 o0 = origin[p_base];
    int rx = 0, ry = 0;
    if (tid < gcount) {
      const int2 o = origin[p_base + tid];
      rx = wrap_mod((long long)o.x - o0.x + ns / 2, ns) - ns / 2;
      ry = wrap_mod((long long)o.y - o0.y + ns / 2, ns) - ns / 2;
    }
    int minx = rx, maxx = rx, miny = ry, maxy = ry;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      minx = min(minx, __shfl_xor(minx, off, 64));
      maxx = max(maxx, __shfl_xor(maxx, off, 64));
      miny = min(miny, __shfl_xor(miny, off, 64));
      maxy = max(maxy, __shfl_xor(maxy, off, 64));
    }
    if (tid < G) {
      offx[tid] = rx - minx;
      offy[tid] = ry - miny;
    }
    if (tid == 0) {
      const int smax = w / 2;
      ginfo[0] = (maxx - minx <= smax && maxy - miny <= smax) ? 0 : 1;
      ginfo[1] = wrap_mod((long long)o0.y + miny, ns);
      ginfo[2] = wrap_mod((long long)o0.x + minx, ns);
      ginfo[3] = w + (maxy - miny);
      ginfo[4] = w + (maxx - minx);
    }
  }
  __syncthreads();
  // the workgroups of a group share its tiles round-robin
  if (ginfo[0] == 0) {
    UnionGeom U{ginfo[1], ginfo[2], ginfo[3], ginfo[4]};
    for (int tile = blockIdx.x; tile * kCTile < U.uy * U.ux; tile += gridDim.x)
      contract_tile<G>(S, act, n_act, alpha, np, p_base, gcount, ns, w, U, tile, offx, offy, -1,
                       smem, window);
  } else {
    // windows too far apart to share: one probe at a time, its window alone
    __shared__ int zero[G];
    for (int g = tid; g < G; g += kCNT) zero[g] = 0;
    __syncthreads();
    for (int tile = blockIdx.x; tile * kCTile < w * w; tile += gridDim.x) {
      for (int g = 0; g < gcount; ++g) {
        const int2 o = origin[p_base + g];
        UnionGeom U{o.y, o.x, w, w};
        contract_tile<G>(S, act, n_act, alpha, np, p_base, gcount, ns, w, U, tile, zero, zero, g,
                         smem, window);
      }
    }
  }
}

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

template <bool CBED>
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
  __shared__ double red[kMaxDet][4];
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
  double acc[kMaxDet];
#pragma unroll
  for (int q = 0; q < kMaxDet; ++q) acc[q] = 0.0;
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) {
    const int kyi = b + R * k2;
    const long long ky = kyi < kW4 / 2 ? kyi : kyi - kW4;
    const long long kk = (long long)f * f * (kx * kx + ky * ky);
    const double I = ((double)v[k2].x * v[k2].x + (double)v[k2].y * v[k2].y) * inv_w2;
#pragma unroll
    for (int q = 0; q < kMaxDet; ++q)
      if (q < bins.n && kk >= bins.lo[q] && kk < bins.hi[q]) acc[q] += I;
  }
#pragma unroll
  for (int q = 0; q < kMaxDet; ++q) {
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
#ifndef PRISM_WD_PREFETCH
#define PRISM_WD_PREFETCH 0  // window kernel: load the next probe during the current one
#endif
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
// walk probes p = blockIdx.x, + gridDim.x, ... (one probe each unless there
// are more than PRISM_WD_GRID); with PRISM_WD_PREFETCH the first row stage
// of the next probe is loaded into registers while the current one is
// transformed (one window fills most of a compute unit's LDS, so this is the
// only overlap there is within a workgroup).
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
                                                            int np,
                                                            const float2* __restrict__ twW,
                                                            const uint16_t* __restrict__ pix,
                                                            BinLists lists,
                                                            double* __restrict__ out,
                                                            float* __restrict__ cbed,
                                                            OutAcc oa) {
  constexpr int NT = wd_nt(W);
  constexpr int NW = NT / 64;
  using Rows = RowBatch<W, W>;
  using Cols = Batch<W, W, W, 0, 1, W, true>;
  using S8 = StageShape<Rows, 8, NT>;
  __shared__ float2 lds[lds_padded(W * W)];
  __shared__ float2 tw[W];
  __shared__ double red[CBED ? 1 : kMaxDet][NW];
  const int tid = threadIdx.x;
  load_twiddles<W, NT>(tw, twW, tid);
  float2 nxt[S8::PER][8];
  auto load = [&](int p) {  // first row stage of window p
    const float2* src = window + (size_t)p * W * W;
#pragma unroll
    for (int q = 0; q < S8::PER; ++q) {
      const int b = tid + q * NT;
      if (!S8::GUARD || b < S8::TOT) {
        int row, j;
        stage_coords<Rows, S8::NB>(b, row, j);
#pragma unroll
        for (int r = 0; r < 8; ++r) nxt[q][r] = src[row * W + j + r * (W / 8)];
      }
    }
  };
  if (PRISM_WD_PREFETCH) load(blockIdx.x);
  const double inv_w2 = 1.0 / ((double)W * (double)W);
#pragma unroll 1
  for (int p = blockIdx.x; p < np; p += gridDim.x) {
    float2 v[S8::PER][8];
    if (!PRISM_WD_PREFETCH) load(p);
#pragma unroll
    for (int q = 0; q < S8::PER; ++q)
#pragma unroll
      for (int r = 0; r < 8; ++r) v[q][r] = nxt[q][r];
    if (PRISM_WD_PREFETCH)
      load(min(p + (int)gridDim.x, np - 1));  // the last round re-reads its own window
    stage_out<Rows, 8, 1, NT, false>(lds, tid, v);
    __syncthreads();
    fft_from<Rows, NT, false, 8>(lds, tw, tid);
    fft_lds<Cols, NT, false>(lds, tw, tid);
    if constexpr (CBED) {
      float* dst = cbed + (size_t)p * W * W;
      for (int e = tid; e < W * W; e += NT) {
        const float2 z = lds[lpad(e)];
        put_out(dst + e, ((double)z.x * z.x + (double)z.y * z.y) * inv_w2, oa);
      }
    } else {
      const int K = lists.off[lists.n];  // chunks of kWdListChunk entries
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
      for (int i = tid; i < lists.n * NW; i += NT) red[i / NW][i % NW] = 0.0;
      __syncthreads();
      const int c0 = (int)((long long)K * wv / NW), c1 = (int)((long long)K * (wv + 1) / NW);
      int j = 0;  // bin of the current chunk (uniform in the wave)
      while (j < lists.n && c0 >= lists.off[j + 1]) ++j;
      double acc = 0.0;
      for (int k0 = c0; k0 < c1; k0 += kWdChunks) {
        int px[kWdChunks];
#pragma unroll
        for (int c = 0; c < kWdChunks; ++c)
          px[c] = k0 + c < c1 ? (int)pix[(size_t)(k0 + c) * kWdListChunk + lane] : (int)kNoPix;
#pragma unroll
        for (int c = 0; c < kWdChunks; ++c) {
          const int k = k0 + c;
          if (k >= c1) break;
          if (k >= lists.off[j + 1]) {  // bin j ends: its wave sum, then the bin of chunk k
            const double sm = wave_sum(acc);
            if (lane == 0) red[j][wv] = sm;
            acc = 0.0;
            do ++j;
            while (k >= lists.off[j + 1]);
          }
          const bool ok = px[c] != (int)kNoPix;
          const float2 z = lds[lpad(ok ? px[c] : 0)];
          const double I = (double)z.x * z.x + (double)z.y * z.y;
          acc += ok ? I : 0.0;
        }
      }
      if (c1 > c0) {
        const double sm = wave_sum(acc);
        if (lane == 0) red[j][wv] = sm;
      }
      __syncthreads();
      if (tid < lists.n) {
        double sm = 0.0;
        for (int w = 0; w < NW; ++w) sm += red[tid][w];
        put_out(out + (size_t)p * lists.n + tid, sm * inv_w2, oa);
      }
    }
    __syncthreads();  // LDS free for the next probe
  }
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int contract_group(int w) { return w >= 128 ? PRISM_CG128 : (w >= 64 ? 32 : 16); }

hipError_t launch_alpha(const double* probe_xy, int p0, int np, const ActiveBeam* act, int n_act,
                        int f, int ns, int w, const ProbeOptics& po, float2* alpha,
                        int2* origin, hipStream_t st) {
  hipLaunchKernelGGL(k_alpha, dim3(blocks_for((size_t)np * n_act, 256)), dim3(256), 0, st,
                     probe_xy, p0, np, act, n_act, f, ns, w, po, alpha, origin);
  return hipGetLastError();
}

int contract_tile_slots(int w) {
  const int own = (w * w + kCTile - 1) / kCTile;  // tiles of one window
  return std::max(1, own / PRISM_CTILES_PER_WG);
}

hipError_t launch_contract(const float2* smatrix, const ActiveBeam* act, int n_act,
                           const float2* alpha, const int2* origin, int np, int ns, int w,
                           int group, float2* window, hipStream_t st) {
  const unsigned groups = (unsigned)((np + group - 1) / group);
  const dim3 grid((unsigned)contract_tile_slots(w), groups);
  switch (group) {
    case 16:
      hipLaunchKernelGGL(k_contract<16>, grid, dim3(kCNT), 0, st, smatrix, act, n_act, alpha,
                         origin, np, ns, w, window);
      break;
    case 32:
      hipLaunchKernelGGL(k_contract<32>, grid, dim3(kCNT), 0, st, smatrix, act, n_act, alpha,
                         origin, np, ns, w, window);
      break;
    case 64:
      hipLaunchKernelGGL(k_contract<64>, grid, dim3(kCNT), 0, st, smatrix, act, n_act, alpha,
                         origin, np, ns, w, window);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int window256_tiles() { return kW4 / 16; }

hipError_t launch_window256(float2* window, int np, const float2* twW, int f,
                            const DetBins& bins, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_window_rows256, dim3((unsigned)((size_t)np * kW4 / kR4)), dim3(256), 0, st,
                     window, twW);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_window_cols256_detect<false>, dim3((unsigned)((size_t)np * window256_tiles())),
                     dim3(256), 0, st, window, twW, f, bins, partial, (float*)nullptr, OutAcc{});
  return hipGetLastError();
}

hipError_t launch_window256_cbed(float2* window, int np, const float2* twW, float* cbed,
                                 OutAcc acc, hipStream_t st) {
  hipLaunchKernelGGL(k_window_rows256, dim3((unsigned)((size_t)np * kW4 / kR4)), dim3(256), 0, st,
                     window, twW);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DetBins none{};
  hipLaunchKernelGGL(k_window_cols256_detect<true>, dim3((unsigned)((size_t)np * window256_tiles())),
                     dim3(256), 0, st, window, twW, 1, none, (double*)nullptr, cbed, acc);
  return hipGetLastError();
}

// Workgroups for the window kernels: one per probe up to PRISM_WD_GRID, then
// each walks several probes.
static unsigned window_grid(int np) { return (unsigned)std::min(np, PRISM_WD_GRID); }

hipError_t launch_window_detect(const float2* window, int np, int w, const float2* twW,
                                const uint16_t* pix, const BinLists& lists, double* out,
                                OutAcc acc, hipStream_t st) {
  if (np <= 0) return hipSuccess;
#define WD(WW)                                                                                  \
  case WW:                                                                                      \
    hipLaunchKernelGGL((k_window_detect<WW, false>), dim3(window_grid(np)), dim3(wd_nt(WW)), 0, \
                       st, window, np, twW, pix, lists, out, (float*)nullptr, acc);             \
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
    default:
      return hipErrorInvalidValue;
  }
#undef WD
  return hipGetLastError();
}

hipError_t launch_window_cbed(const float2* window, int np, int w, const float2* twW,
                              float* cbed, OutAcc acc, hipStream_t st) {
  if (np <= 0) return hipSuccess;
  BinLists none{};
#define WC(WW)                                                                                 \
  case WW:                                                                                     \
    hipLaunchKernelGGL((k_window_detect<WW, true>), dim3(window_grid(np)), dim3(wd_nt(WW)), 0, \
                       st, window, np, twW, (const uint16_t*)nullptr, none, (double*)nullptr,  \
                       cbed, acc);                                                             \
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
    default:
      return hipErrorInvalidValue;
  }
#undef WC
  return hipGetLastError();
}

}  // namespace prism
