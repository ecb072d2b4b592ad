// Multislice kernels (Eqs. 3-5) shared by the PRISM S-matrix build (Fig. 1c)
// and by conventional multislice STEM.
//
// One slice step psi <- iFFT2( FFT2(psi t_p) P_p M ) is split into two
// HBM passes over the compact state X(y, kx) (layout in kernels.hpp):
//   row pass    : X -> iFFT_x -> * t_p / n -> FFT_x -> keep |kx| < n/4 -> X'
//   column pass : X' -> FFT_y -> * P_p(kx) P_p(ky) M / n -> iFFT_y -> X''
// P_p is separable, so it comes from a 1D table per slice; M is the
// half-band anti-aliasing aperture kx^2 + ky^2 < (n/4)^2. Each pass reads
// and writes n^2/2 complex values per wave.
#include <algorithm>

#include "fft_lds.hpp"
#include "fft_reg.hpp"
#include "kernels.hpp"

namespace prism {

namespace {

// Launch shapes (tuned on MI355X; overridable at build time).
#ifndef PRISM_ROW_ELEMS
#define PRISM_ROW_ELEMS 2048   // complex values per row-pass workgroup
#endif
#ifndef PRISM_COL_E
#define PRISM_COL_E 8          // complex values per column-pass thread
#endif
#ifndef PRISM_COL_WPE
#define PRISM_COL_WPE 1        // minimum waves per SIMD for the column pass
#endif

constexpr int kRowNT = PRISM_ROW_ELEMS / 8;

// Largest power of two p with p n <= cap (at least 1): rows per workgroup
// that divide every wave's n rows (n = 2^k, 3 2^k or 9 2^k).
__host__ __device__ constexpr int pow2_rows(int n, int cap) {
  return 2 * n <= cap ? 2 * pow2_rows(2 * n, cap) : 1;
}
__host__ __device__ constexpr int row_nseq(int n) { return pow2_rows(n, PRISM_ROW_ELEMS); }
__host__ __device__ constexpr int col_tc(int n) { return 8; }
__host__ __device__ constexpr int col_nt(int n) {
  return (col_tc(n) * n / PRISM_COL_E) < 64
             ? 64
             : (col_tc(n) * n / PRISM_COL_E > 1024 ? 1024 : col_tc(n) * n / PRISM_COL_E);
}
__host__ __device__ constexpr int ext_nseq(int n) { return pow2_rows(n, 4096); }

// Map launch order onto tiles so that consecutive tiles run on the same
// XCD (workgroups are dealt to the 8 XCDs round-robin) and share its L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  if ((nb & 7) != 0) return bid;
  return (bid & 7) * (nb >> 3) + (bid >> 3);
}

__device__ __forceinline__ int signed_k(int idx, int n) { return idx < n / 2 ? idx : idx - n; }

// ---------------------------------------------------------------------------
__global__ void k_twiddles(float2* tw, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L) {
    double s, c;
    sincospi(-2.0 * (double)i / (double)L, &s, &c);
    tw[i] = make_float2((float)c, (float)s);
  }
}

// tw2[m][j] = exp(-2 pi i j m / n) for j, m < R, n = R^2 (four-step passes).
__global__ void k_twiddles2(float2* tw2, int R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R * R) {
    const int m = i / R, j = i % R;
    double s, c;
    sincospi(-2.0 * (double)(j * m) / (double)(R * R), &s, &c);
    tw2[i] = make_float2((float)c, (float)s);
  }
}

// t_p = exp(i phi_p) / n, the 1/n belonging to the row pass' inverse FFT.
__global__ void k_transmission(const float* __restrict__ phase, float2* __restrict__ trans,
                               size_t count, float scale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    double s, c;
    sincos((double)phase[i], &s, &c);
    trans[i] = make_float2((float)(c * scale), (float)(s * scale));
  }
}

__global__ void k_prop_lut(float2* lut, int n, int H, const double* __restrict__ thick, double lam,
                           double dq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * H) return;
  const int p = i / n, idx = i % n;
  const double k = (double)signed_k(idx, n);
  double s, c;
  sincospi(-lam * thick[p] * (k * dq) * (k * dq), &s, &c);
  lut[i] = make_float2((float)c, (float)s);
}

// Tilted plane wave exp(2 pi i (m f x + n f y) / n) in compact form:
// X(y, kx) = n exp(2 pi i ((n f y) mod n) / n) at kx = m f, zero elsewhere.
__global__ void k_beam_init(float2* __restrict__ state, const int32_t* __restrict__ mn, int b0,
                            int nb, int n, int f, const float2* __restrict__ twN) {
  const int h2 = n / 2;
  const size_t total = (size_t)nb * n * h2;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int w = (int)(i / ((size_t)n * h2));
  const int rem = (int)(i % ((size_t)n * h2));
  const int y = rem / h2, jj = rem % h2;
  const int m = mn[2 * (b0 + w)], nn = mn[2 * (b0 + w) + 1];
  const int kx = m * f;
  const int jj0 = kx >= 0 ? kx : kx + h2;
  float2 v = make_float2(0.f, 0.f);
  if (jj == jj0) {
    long long idx = ((long long)nn * f * y) % n;
    if (idx < 0) idx += n;
    const float2 t = twN[idx];  // exp(-2 pi i idx / n)
    v = make_float2(t.x * (float)n, -t.y * (float)n);
  }
  state[i] = v;
}

// ---------------------------------------------------------------------------
// Row pass: NSEQ rows of length n per workgroup (PRISM_ROW_ELEMS complex in
// LDS). The inverse x-transform runs 8, 8^MID, RL and the forward one
// RL, 8^MID, 8 (PairedPlan): the inverse's first stage reads the compact row
// straight from HBM (its inputs at |kx| >= n/4 are zero), its last stage
// stays in registers, is multiplied by t_p / n and feeds the forward's first
// stage, and the forward's last stage stores only the kept half band.
// WT: each wave w reads its own transmission wtrans[w] + soff (waves of
// several specimens in one launch); otherwise every wave reads trans.
template <int N, bool WT>
__global__ __launch_bounds__(kRowNT) void k_row_pass(float2* __restrict__ state,
                                                     const float2* __restrict__ trans,
                                                     const float2* const* __restrict__ wtrans,
                                                     size_t soff,
                                                     const float2* __restrict__ twN) {
  constexpr int NT = kRowNT;
  constexpr int NSEQ = row_nseq(N);
  constexpr int H2 = N / 2, E8 = N / 8;
  using B = RowBatch<N, NSEQ>;
  using PP = PairedPlan<N>;
  constexpr int RL = PP::RL, NSL = N / PP::RL;
  using S8 = StageShape<B, 8, NT>;
  using SL = StageShape<B, RL, NT>;
  __shared__ float2 lds[lds_padded(NSEQ * N)];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  const size_t row0 = (size_t)blockIdx.x * NSEQ;
  load_twiddles<N, NT>(tw, twN, tid);
  {
    // inverse, first stage (span 1): inputs j + r n/8, nonzero for r in {0,1,6,7}
    float2 v[S8::PER][8];
#pragma unroll
    for (int p = 0; p < S8::PER; ++p) {
      const int b = tid + p * NT;
      v[p][2] = v[p][3] = v[p][4] = v[p][5] = make_float2(0.f, 0.f);
      if (S8::GUARD && b >= S8::TOT) continue;  // no butterfly (stage_out skips it too)
      int sq, j;
      stage_coords<B, S8::NB>(b, sq, j);
      const float2* src = state + (row0 + sq) * H2 + j;
      v[p][0] = src[0];
      v[p][1] = src[E8];
      v[p][6] = src[2 * E8];
      v[p][7] = src[3 * E8];
    }
    stage_out<B, 8, 1, NT, true>(lds, tid, v);
  }
  __syncthreads();
  fft_radix8_run<B, NT, true, 8, PP::MID>(lds, tw, tid);
  float2 v[SL::PER][RL];
  stage_in<B, RL, NSL, NT, true>(lds, tw, tid, v);
#pragma unroll
  for (int p = 0; p < SL::PER; ++p) {
    const int b = tid + p * NT;
    if (SL::GUARD && b >= SL::TOT) continue;
    int sq, j;
    stage_coords<B, SL::NB>(b, sq, j);
    dft<RL, true>(v[p]);
    const float2* tb = WT ? wtrans[(row0 + sq) / N] + soff : trans;
    const float2* t = tb + (size_t)((row0 + sq) % (size_t)N) * N + j;
#pragma unroll
    for (int r = 0; r < RL; ++r) v[p][r] = cmul(v[p][r], t[r * NSL]);
  }
  __syncthreads();
  stage_out<B, RL, 1, NT, false>(lds, tid, v);
  __syncthreads();
  fft_radix8_run<B, NT, false, RL, PP::MID>(lds, tw, tid);
  {
    // forward, last stage (span n/8): outputs j + r n/8, kept for r in {0,1,6,7}
    float2 w[S8::PER][8];
    stage_in<B, 8, E8, NT, false>(lds, tw, tid, w);
#pragma unroll
    for (int p = 0; p < S8::PER; ++p) {
      const int b = tid + p * NT;
      if (S8::GUARD && b >= S8::TOT) continue;
      int sq, j;
      stage_coords<B, S8::NB>(b, sq, j);
      dft8<false>(w[p]);
      float2* dst = state + (row0 + sq) * H2 + j;
      dst[0] = w[p][0];
      dst[E8] = w[p][1];
      dst[2 * E8] = w[p][6];
      dst[3 * E8] = w[p][7];
    }
  }
}

// ---------------------------------------------------------------------------
// Four-step row pass for n = R^2 (R = 16, 32). Row element x = R a + b sits
// with lane b (R lanes per row, 64 / R rows per wave):
//   inverse: lane b transforms over a (only a < R/4 and a >= 3R/4 are
//            nonzero: the compact half band), twiddles by w_n^{-bc}, one LDS
//            transpose, lane c transforms over b -> psi(c + R d);
//   t_p / n multiplies psi in registers;
//   forward: lane c transforms over d (the same registers), twiddles by
//            w_n^{ce}, one LDS transpose, lane e transforms over c and
//            stores the outputs e + R g with |kx| < n/4.
// Each wave owns its LDS rows, so the transposes need only wave-level
// ordering. Each lane keeps its R - 1 twiddles w_n^{jc} in registers for the
// whole kernel (no table reads between the transforms). A workgroup walks
// `iters` row groups; each wave loads the next row's inputs and the current
// row's t_p while it computes.

// Raw buffer resource over count complex values at p (gfx9 word 3), and
// 8-byte loads / stores at vector offset voff + scalar offset soff (bytes).
// Accesses past the resource read zero / are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const float2* p, int count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(p), 0, count * 8, 0x00020000);
}
typedef int int2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff,
                                          float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(int2v, v), r, voff, soff, 0);
}

// Orders LDS accesses of one wave (compiler barrier; LDS executes a wave's
// instructions in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R, bool WT>
__global__ __launch_bounds__(256) void k_row_pass4(float2* __restrict__ state,
                                                   const float2* __restrict__ trans,
                                                   const float2* const* __restrict__ wtrans,
                                                   size_t soff,
                                                   const float2* __restrict__ tw2, int iters) {
  constexpr int N = R * R, H2 = N / 2, Q = R / 4, LS = R + 1;
  constexpr int RPW = 64 / R;             // rows per wave
  constexpr int RS = R * LS + 8;          // LDS row stride (float2)
  constexpr int GROUP = 4 * RPW;          // rows per workgroup iteration
  __shared__ float2 lds[4 * RPW * RS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = lane % R, rw = lane / R;
  float2* L = lds + (wv * RPW + rw) * RS;
  const size_t row_base = (size_t)blockIdx.x * (GROUP * iters) + wv * RPW + rw;

  float2 s[2 * Q];  // compact inputs of the next row: a < Q, then a >= R - Q
  // Buffer loads from the workgroup's first row; live == false gives a
  // zero-length resource (zeros, no memory traffic).
  const float2* wg_rows = state + (size_t)blockIdx.x * (GROUP * iters) * H2;
  const unsigned lane_off = (unsigned)(((wv * RPW + rw) * H2 + j) * 8);
  auto load_src = [&](int it, bool live) {
    const __amdgpu_buffer_rsrc_t rs = wave_rsrc(wg_rows, live ? GROUP * iters * H2 : 0);
    const int soff = it * GROUP * H2 * 8;
#pragma unroll
    for (int a = 0; a < Q; ++a) s[a] = buf_load(rs, lane_off, soff + R * a * 8);
#pragma unroll
    for (int a = 0; a < Q; ++a) s[Q + a] = buf_load(rs, lane_off, soff + (R * (R - Q + a) - H2) * 8);
  };
  load_src(0, true);
  // this lane's four-step twiddles w_n^{jc}, c = 1 .. R-1 (the same values
  // serve the inverse, conjugated, and the forward transform), held in
  // registers for the whole loop
  float2 tw[R - 1];
#pragma unroll
  for (int c = 1; c < R; ++c) tw[c - 1] = tw2[c * R + j];
  // wait here for the first row and the twiddles (s_waitcnt vmcnt(0)) so
  // that the loop head
  // carries no pending load and never waits for the previous row's stores
  __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
    const size_t row = row_base + (size_t)it * GROUP;
    float2 v[R];
#pragma unroll
    for (int a = 0; a < R; ++a)
      v[a] = a < Q ? s[a] : (a >= R - Q ? s[a - (R - 2 * Q)] : make_float2(0.f, 0.f));
    // Next row's inputs first, then this row's t_p: both are waited for
    // together at the t_p product, after the inverse transform, so no load
    // is still pending (and no store waited for) at the top of the loop.
    load_src(min(it + 1, iters - 1), it + 1 < iters);
    float2 tt[R];
    {
      const float2* tb = WT ? wtrans[row / N] + soff : trans;
      const float2* t = tb + (row & (size_t)(N - 1)) * N + j;
#pragma unroll
      for (int d = 0; d < R; ++d) tt[d] = t[R * d];
    }
    dft_reg<R, true>(v);
#pragma unroll
    for (int c = 0; c < R; ++c) L[c * LS + j] = c ? cmulc(v[c], tw[c - 1]) : v[c];
    wave_sync();
#pragma unroll
    for (int b = 0; b < R; ++b) v[b] = L[j * LS + b];
    dft_reg<R, true>(v);
#pragma unroll
    for (int d = 0; d < R; ++d) v[d] = cmul(v[d], tt[d]);
    dft_reg<R, false>(v);
    wave_sync();
#pragma unroll
    for (int e = 0; e < R; ++e) L[e * LS + j] = e ? cmul(v[e], tw[e - 1]) : v[e];
    wave_sync();
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[j * LS + c];
    dft_reg<R, false>(v);
    float2* dst = state + row * H2 + j;
#pragma unroll
    for (int g = 0; g < R; ++g) {
      if (g < Q) dst[R * g] = v[g];
      else if (g >= R - Q) dst[R * g - H2] = v[g];
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Four-step column pass for n = R^2 over tiles of TC adjacent compact
// columns (TC R threads); lane (b, c) = (tid / TC, tid % TC), so each load or
// store instruction covers TC contiguous columns of 64 / TC rows.
//   forward : lane (b, c) transforms y = R a + b over a, twiddles by
//             w_n^{b k1}, LDS transpose, lane (k1, c) transforms over b and
//             keeps ky = k1 + R k2 with |ky| < n/4 (the rest is cut by M);
//   P_p(kx) P_p(ky) M / n in registers;
//   inverse : lane (k1, c) transforms over k2 (inputs outside the half band
//             are zero), twiddles by w_n^{-k1 m1}, LDS transpose, lane
//             (m1, c) transforms over k1 and stores y = m1 + R m2.
// A workgroup walks `iters` tiles, loading the next tile while it
// computes the current one.
#ifndef PRISM_COL4_TC32
#define PRISM_COL4_TC32 16   // columns per tile at n = 1024
#endif

template <int R, int TC>
__global__ __launch_bounds__(TC * R) __attribute__((amdgpu_waves_per_eu(2))) void k_col_pass4(float2* __restrict__ state,
                                                   const float2* __restrict__ prop,
                                                   const float2* __restrict__ tw2, int iters) {
  constexpr int N = R * R, H2 = N / 2, Q = R / 4, LS = R + 1;
  constexpr int NT = TC * R;
  constexpr int TILES = H2 / TC;         // tiles per wave
  constexpr int CS = R * LS + 16 / TC;   // LDS column stride (float2): the TC
                                         // columns of a 16-lane group hit
                                         // distinct banks
  __shared__ float2 twl[R * R];
  __shared__ float2 pyl[H2];  // P_p(ky) for |ky| < n/4, compact order
  __shared__ float2 lds[TC * CS];
  const int tid = threadIdx.x, c = tid % TC, b = tid / TC;
  for (int i = tid; i < R * R; i += NT) twl[i] = tw2[i];
  for (int i = tid; i < H2; i += NT) pyl[i] = prop[i < H2 / 2 ? i : i + H2];
  float2* L = lds + c * CS;
  const float2* twb = twl + b;
  const float inv_n = 1.0f / (float)N;

  // Buffer accesses: one wave function per resource, lane (b, c) at a fixed
  // vector byte offset, the row and tile offsets in scalar registers.
  const unsigned lane_off = (unsigned)(b * H2 + c) * 8u;
  float2 s[R];  // next tile's column elements y = R a + b
  // live == false: a zero-length resource, the loads return zeros and
  // touch no memory (keeps the instruction stream of every iteration alike)
  auto load_tile = [&](int tile, bool live) {
    const int w = tile / TILES, c0 = (tile % TILES) * TC;
    const __amdgpu_buffer_rsrc_t rs =
        wave_rsrc(state + (size_t)w * N * H2, live ? N * H2 : 0);
#pragma unroll
    for (int a = 0; a < R; ++a) s[a] = buf_load(rs, lane_off, (c0 + R * a * H2) * 8);
  };
  // Iteration it handles tile it * gridDim.x + g, with g the XCD-grouped
  // workgroup index: workgroups resident on one XCD at the same time take
  // adjacent tiles, which share the 128-byte lines of every row.
  const int g = xcd_tile(blockIdx.x, gridDim.x), nwg = gridDim.x;
  load_tile(g, true);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): no load pending at the loop head
  __syncthreads();
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
    const int tile = it * nwg + g;
    const int w = tile / TILES, c0 = (tile % TILES) * TC;
    float2 v[R];
#pragma unroll
    for (int a = 0; a < R; ++a) v[a] = s[a];
    // the next tile is in flight during this one
    load_tile(min(it + 1, iters - 1) * nwg + g, it + 1 < iters);
    dft_reg<R, false>(v);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) L[k1 * LS + b] = v[k1];
    __syncthreads();
    const int jj = c0 + c;
    const int kx = jj < H2 / 2 ? jj : jj - H2;
    // P_p(kx) from the same LDS table as P_p(ky) (compact index jj): a
    // global load here would be waited for together with the next tile's
    // loads (vector memory counts complete in order)
    const float2 px = cscale(pyl[jj], inv_n);
    // the twiddle w_n^{bb k1} is applied on the reading side (the table is
    // symmetric, so the reading lane k1 = b indexes it by bb): the element
    // and twiddle reads go out together instead of one twiddle read waited
    // for per LDS write
    {
      float2 tw[R - 1];
#pragma unroll
      for (int bb = 0; bb < R; ++bb) v[bb] = L[b * LS + bb];
#pragma unroll
      for (int bb = 1; bb < R; ++bb) tw[bb - 1] = twb[bb * R];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int bb = 1; bb < R; ++bb) v[bb] = cmul(v[bb], tw[bb - 1]);
    }
    dft_reg<R, false>(v);  // lane (k1 = b, c): ky index b + R k2
    {
      // P_p(ky) of the kept rows, read together; the band limit is a select
      // on the computed product (no branch per element)
      float2 p2[2 * Q];
#pragma unroll
      for (int k2 = 0; k2 < 2 * Q; ++k2) {
        const int kyi = b + R * (k2 < Q ? k2 : k2 + R - 2 * Q);
        p2[k2] = pyl[k2 < Q ? kyi : kyi - H2];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k2 = 0; k2 < R; ++k2) {
        if (k2 < Q || k2 >= R - Q) {
          const int kyi = b + R * k2;
          const int ky = kyi < H2 ? kyi : kyi - N;
          float2 m = cmul(cmul(v[k2], px), p2[k2 < Q ? k2 : k2 - (R - 2 * Q)]);
          asm volatile("" : "+v"(m.x), "+v"(m.y));
          const bool keep = 16 * (kx * kx + ky * ky) < N * N;
          v[k2] = make_float2(keep ? m.x : 0.f, keep ? m.y : 0.f);
        } else {
          v[k2] = make_float2(0.f, 0.f);
        }
      }
    }
    dft_reg<R, true>(v);  // over k2 -> m1
    __syncthreads();
#pragma unroll
    for (int m1 = 0; m1 < R; ++m1) L[m1 * LS + b] = v[m1];
    __syncthreads();
    {
      float2 tw[R - 1];
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) v[k1] = L[b * LS + k1];
#pragma unroll
      for (int k1 = 1; k1 < R; ++k1) tw[k1 - 1] = twb[k1 * R];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k1 = 1; k1 < R; ++k1) v[k1] = cmulc(v[k1], tw[k1 - 1]);
    }
    dft_reg<R, true>(v);  // lane (m1 = b, c): y = b + R m2
    const __amdgpu_buffer_rsrc_t rd = wave_rsrc(state + (size_t)w * N * H2, N * H2);
#pragma unroll
    for (int m2 = 0; m2 < R; ++m2) buf_store(rd, lane_off, (c0 + R * m2 * H2) * 8, v[m2]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Column pass over a tile of TC adjacent compact columns, held [y][c]. The
// forward y-transform reads straight from HBM, its last stage stays in
// registers for the propagator and band limit, and the inverse's last stage
// stores straight to HBM (PairedPlan order, as in the row pass).
// DETECT: last multislice slice; instead of the inverse transform, form
// I = |Psi|^2 / n^2 and write per-tile detector partial sums.
template <int N, bool DETECT>
__global__ __launch_bounds__(col_nt(N)) __attribute__((amdgpu_waves_per_eu(PRISM_COL_WPE)))
void k_col_pass(float2* __restrict__ state, const float2* __restrict__ prop,
                const float2* __restrict__ twN, DetBins bins, double* __restrict__ partial) {
  constexpr int TC = col_tc(N), NT = col_nt(N);
  constexpr int H2 = N / 2, Q = N / 4, E8 = N / 8;
  constexpr int TILES = H2 / TC;
  constexpr int NW = NT / 64;
  using B = Batch<N, TC, TC, 0, 1, TC, true>;
  using PP = PairedPlan<N>;
  constexpr int RL = PP::RL, NSL = N / PP::RL;
  using S8 = StageShape<B, 8, NT>;
  using SL = StageShape<B, RL, NT>;
  __shared__ float2 lds[lds_padded(TC * N)];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int w = tile / TILES, c0 = (tile % TILES) * TC;
  float2* base = state + (size_t)w * N * H2 + c0;
  load_twiddles<N, NT>(tw, twN, tid);
  {
    float2 v[S8::PER][8];
#pragma unroll
    for (int p = 0; p < S8::PER; ++p) {
      const int b = tid + p * NT;
      if (S8::GUARD && b >= S8::TOT) continue;  // no butterfly (stage_out skips it too)
      int c, j;
      stage_coords<B, S8::NB>(b, c, j);
#pragma unroll
      for (int r = 0; r < 8; ++r) v[p][r] = base[(size_t)(j + r * E8) * H2 + c];
    }
    stage_out<B, 8, 1, NT, false>(lds, tid, v);
  }
  __syncthreads();
  fft_radix8_run<B, NT, false, 8, PP::MID>(lds, tw, tid);
  float2 v[SL::PER][RL];
  stage_in<B, RL, NSL, NT, false>(lds, tw, tid, v);
  const float inv_n = 1.0f / (float)N;
#pragma unroll
  for (int p = 0; p < SL::PER; ++p) {
    const int b = tid + p * NT;
    if (SL::GUARD && b >= SL::TOT) continue;
    int c, j;
    stage_coords<B, SL::NB>(b, c, j);
    dft<RL, false>(v[p]);
    const int jj = c0 + c;
    const int kx = jj < Q ? jj : jj - H2;
    const float2 px = prop[kx < 0 ? kx + N : kx];
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int yi = j + r * NSL;
      const int ky = signed_k(yi, N);
      const int k2 = kx * kx + ky * ky;
      if (16 * k2 < N * N) {
        float2 z = cmul(cmul(v[p][r], px), prop[yi]);
        v[p][r] = DETECT ? z : cscale(z, inv_n);
      } else {
        v[p][r] = make_float2(0.f, 0.f);
      }
    }
  }
  if constexpr (!DETECT) {
    __syncthreads();
    stage_out<B, RL, 1, NT, true>(lds, tid, v);
    __syncthreads();
    fft_radix8_run<B, NT, true, RL, PP::MID>(lds, tw, tid);
    float2 u[S8::PER][8];
    stage_in<B, 8, E8, NT, true>(lds, tw, tid, u);
#pragma unroll
    for (int p = 0; p < S8::PER; ++p) {
      const int b = tid + p * NT;
      if (S8::GUARD && b >= S8::TOT) continue;
      int c, j;
      stage_coords<B, S8::NB>(b, c, j);
      dft8<true>(u[p]);
#pragma unroll
      for (int r = 0; r < 8; ++r) base[(size_t)(j + r * E8) * H2 + c] = u[p][r];
    }
  } else {
    __shared__ double red[8][NW];
    const double inv_n2 = 1.0 / ((double)N * (double)N);
    for (int j0 = 0; j0 < bins.n; j0 += 8) {
      double acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
#pragma unroll
      for (int p = 0; p < SL::PER; ++p) {
        const int b = tid + p * NT;
        if (SL::GUARD && b >= SL::TOT) continue;
        int c, j;
        stage_coords<B, SL::NB>(b, c, j);
        const int jj = c0 + c;
        const int kx = jj < Q ? jj : jj - H2;
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int ky = signed_k(j + r * NSL, N);
          const int k2 = kx * kx + ky * ky;
          const double I = ((double)v[p][r].x * v[p][r].x + (double)v[p][r].y * v[p][r].y) * inv_n2;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int jb = j0 + q;
            if (jb < bins.n && k2 >= bins.lo[jb] && k2 < bins.hi[jb]) acc[q] += I;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double sum = wave_sum(acc[q]);
        if ((tid & 63) == 0) red[q][tid >> 6] = sum;
      }
      __syncthreads();
      if (tid < 8 && j0 + tid < bins.n) {
        double sum = 0.0;
        for (int wv = 0; wv < NW; ++wv) sum += red[tid][wv];
        partial[((size_t)w * TILES + (tile % TILES)) * bins.n + j0 + tid] = sum;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Incident multislice probe, built per compact column in Fourier space and
// brought to X(y, kx) by an inverse FFT along y:
//   X0(y, kx) = norm * sum_ky A e^{-i chi} e^{-2 pi i q.(r0 - s)} e^{2 pi i ky y / n}
// with norm = 1 / sqrt(N_A), chi at k - k_t and s the tilt's entrance offset.
// The aperture comes as one kx interval per row (decided on the host).
// Phases are evaluated in FP64.
template <int N>
__global__ __launch_bounds__(col_nt(N)) void k_probe_init(float2* __restrict__ state,
                                                          const double* __restrict__ probe_xy,
                                                          int p0, ProbeOptics po,
                                                          const int2* __restrict__ aper,
                                                          const float2* __restrict__ twN) {
  constexpr int TC = col_tc(N), NT = col_nt(N);
  constexpr int H2 = N / 2, Q = N / 4;
  constexpr int TILES = H2 / TC;
  using B = Batch<N, TC, TC, 0, 1, TC, true>;
  __shared__ float2 lds[lds_padded(TC * N)];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int w = tile / TILES, c0 = (tile % TILES) * TC;
  const double x0 = probe_xy[2 * (size_t)(p0 + w)] - po.sx;
  const double y0 = probe_xy[2 * (size_t)(p0 + w) + 1] - po.sy;
  load_twiddles<N, NT>(tw, twN, tid);
  const double dq2 = po.dq * po.dq;
  for (int e = tid; e < TC * N; e += NT) {
    const int y = e / TC, c = e % TC;
    const int jj = c0 + c;
    const int kx = jj < Q ? jj : jj - H2;
    const int ky = signed_k(y, N);
    const int2 row = aper[ky + N / 2];
    float2 v = make_float2(0.f, 0.f);
    if (kx >= row.x && kx <= row.y) {
      const double dx = (double)kx - po.ktx, dy = (double)ky - po.kty;
      const double q2 = (dx * dx + dy * dy) * dq2;
      double t = -(0.5 * po.lam * q2 * po.C1 + 0.25 * po.lam * po.lam * po.lam * q2 * q2 * po.C3) -
                 ((double)kx * x0 + (double)ky * y0) * po.dq;
      t -= floor(t);
      double s, co;
      sincospi(2.0 * t, &s, &co);
      v = make_float2((float)(co * po.norm), (float)(s * po.norm));
    }
    lds[lpad(e)] = v;
  }
  __syncthreads();
  fft_lds<B, NT, true>(lds, tw, tid);
  float2* base = state + (size_t)w * N * H2 + c0;
  for (int e = tid; e < TC * N; e += NT) {
    const int y = e / TC, c = e % TC;
    base[(size_t)y * H2 + c] = lds[lpad(e)];
  }
}

// ---------------------------------------------------------------------------
// Quarter-size exit wave: S(i', j') = psi_H(2 i', 2 j')
//   = (1/n) sum_kx X(2 j', kx) exp(2 pi i kx i' / (n/2)),
// an n/2-point inverse FFT of the even compact rows (already in n/2
// fftfreq order).
template <int N>
__global__ __launch_bounds__(256) void k_extract(const float2* __restrict__ state,
                                                 float2* __restrict__ S,
                                                 const float2* __restrict__ twH) {
  constexpr int NT = 256;
  constexpr int H2 = N / 2;
  constexpr int NSEQ = ext_nseq(N);
  using B = RowBatch<H2, NSEQ>;
  __shared__ float2 lds[lds_padded(NSEQ * H2)];
  __shared__ float2 tw[H2];
  const int tid = threadIdx.x;
  const size_t g0 = (size_t)blockIdx.x * NSEQ;
  load_twiddles<H2, NT>(tw, twH, tid);
  for (int e = tid; e < NSEQ * H2; e += NT) {
    const int s = e / H2, i = e % H2;
    const size_t g = g0 + s;
    const size_t w = g / H2, jp = g % H2;
    lds[lpad(e)] = state[(w * N + 2 * jp) * H2 + i];
  }
  __syncthreads();
  fft_lds<B, NT, true>(lds, tw, tid);
  const float inv_n = 1.0f / (float)N;
  for (int e = tid; e < NSEQ * H2; e += NT) {
    const int s = e / H2, i = e % H2;
    S[(g0 + s) * H2 + i] = cscale(lds[lpad(e)], inv_n);
  }
}

__global__ void k_reduce_partials(const double* __restrict__ partial, int nwaves, int tiles,
                                  int n_det, double* __restrict__ out, OutAcc acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nwaves * n_det) return;
  const int w = i / n_det, j = i % n_det;
  double s = 0.0;
  for (int t = 0; t < tiles; ++t) s += partial[((size_t)w * tiles + t) * n_det + j];
  put_out(out + i, s, acc);
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers (sizes are validated by the host plan before any call).

hipError_t launch_twiddles(float2* tw, int L, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(L, 256)), dim3(256), 0, st, tw, L);
  return hipGetLastError();
}

hipError_t launch_transmission(const float* phase, float2* trans, size_t count, float scale,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_transmission, dim3(blocks_for(count, 256)), dim3(256), 0, st, phase, trans,
                     count, scale);
  return hipGetLastError();
}

hipError_t launch_prop_lut(float2* lut, int n, int H, const double* thick_dev, double lam,
                           double dq, hipStream_t st) {
  hipLaunchKernelGGL(k_prop_lut, dim3(blocks_for((size_t)n * H, 256)), dim3(256), 0, st, lut, n,
                     H, thick_dev, lam, dq);
  return hipGetLastError();
}

hipError_t launch_beam_init(float2* state, const int32_t* beams_mn, int b0, int nb, int n, int f,
                            const float2* twN, hipStream_t st) {
  const size_t total = (size_t)nb * n * (n / 2);
  hipLaunchKernelGGL(k_beam_init, dim3(blocks_for(total, 256)), dim3(256), 0, st, state, beams_mn,
                     b0, nb, n, f, twN);
  return hipGetLastError();
}

#define PRISM_DISPATCH_N(n, CALL) \
  switch (n) {                    \
    case 128: CALL(128); break;   \
    case 192: CALL(192); break;   \
    case 256: CALL(256); break;   \
    case 384: CALL(384); break;   \
    case 512: CALL(512); break;   \
    case 576: CALL(576); break;   \
    case 768: CALL(768); break;   \
    case 1024: CALL(1024); break; \
    case 1152: CALL(1152); break; \
    case 1536: CALL(1536); break; \
    case 2048: CALL(2048); break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_twiddles2(float2* tw2, int n, hipStream_t st) {
  const int R = four_step_radix(n);
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_twiddles2, dim3(blocks_for((size_t)R * R, 256)), dim3(256), 0, st, tw2, R);
  return hipGetLastError();
}

int four_step_radix(int n) { return n == 1024 ? 32 : (n == 256 ? 16 : 0); }

// Largest power of two <= maxit dividing units with units / it >= min_wgs
// (1 if none).
static int pick_iters(int units, int maxit, int min_wgs) {
  int it = maxit;
  while (it > 1 && (units % it != 0 || units / it < min_wgs)) it /= 2;
  return it;
}

hipError_t launch_row_pass(float2* state, int nwaves, int n, const float2* trans_p,
                           const float2* twN, const float2* tw2, const LaunchTuning& tune,
                           hipStream_t st, const float2* const* wtrans, size_t soff) {
  // row groups of 4 waves x 64/R rows; the iteration count is the largest
  // power of two (up to tune.row_iters) that divides them and still leaves
  // tune.row_min_wg workgroups
  const bool wt = wtrans != nullptr;
  if (n == 1024 || n == 256) {
    const int R = n == 1024 ? 32 : 16;
    const int groups = nwaves * n / (4 * 64 / R);
    const int it = pick_iters(groups, tune.row_iters, tune.row_min_wg);
    const dim3 grid((unsigned)(groups / it));
#define ROW4(RR, WW)                                                                            \
  hipLaunchKernelGGL((k_row_pass4<RR, WW>), grid, dim3(256), 0, st, state, trans_p, wtrans, soff, \
                     tw2, it)
    if (R == 32) {
      if (wt) ROW4(32, true); else ROW4(32, false);
    } else {
      if (wt) ROW4(16, true); else ROW4(16, false);
    }
#undef ROW4
    return hipGetLastError();
  }
#define ROW(NN)                                                                                 \
  if (wt)                                                                                       \
    hipLaunchKernelGGL((k_row_pass<NN, true>),                                                  \
                       dim3((unsigned)((size_t)nwaves * NN / row_nseq(NN))), dim3(kRowNT), 0,   \
                       st, state, trans_p, wtrans, soff, twN);                                  \
  else                                                                                          \
    hipLaunchKernelGGL((k_row_pass<NN, false>),                                                 \
                       dim3((unsigned)((size_t)nwaves * NN / row_nseq(NN))), dim3(kRowNT), 0,   \
                       st, state, trans_p, wtrans, soff, twN)
  PRISM_DISPATCH_N(n, ROW)
#undef ROW
  return hipGetLastError();
}

int col_tiles(int n) { return (n / 2) / col_tc(n); }

hipError_t launch_col_pass(float2* state, int nwaves, int n, const float2* prop_p,
                           const float2* twN, const float2* tw2, const LaunchTuning& tune,
                           hipStream_t st) {
  // tiles per launch: nwaves x (n/2) / TC, walked up to tune.col_iters at a
  // time while tune.col_min_wg workgroups remain
  if (n == 1024) {
    constexpr int TC = PRISM_COL4_TC32, TPW = 512 / TC;
    const int tiles = nwaves * TPW;
    const int it = pick_iters(tiles, tune.col_iters, tune.col_min_wg);
    hipLaunchKernelGGL((k_col_pass4<32, TC>), dim3((unsigned)(tiles / it)), dim3(TC * 32), 0, st,
                       state, prop_p, tw2, it);
    return hipGetLastError();
  }
  if (n == 256) {
    const int tiles = nwaves * 8, it = pick_iters(tiles, tune.col_iters, tune.col_min_wg);
    hipLaunchKernelGGL((k_col_pass4<16, 16>), dim3((unsigned)(tiles / it)), dim3(256), 0, st,
                       state, prop_p, tw2, it);
    return hipGetLastError();
  }
  DetBins none{};
#define COL(NN)                                                                                  \
  hipLaunchKernelGGL((k_col_pass<NN, false>), dim3((unsigned)(nwaves * col_tiles(NN))),          \
                     dim3(col_nt(NN)), 0, st, state, prop_p, twN, none, (double*)nullptr)
  PRISM_DISPATCH_N(n, COL)
#undef COL
  return hipGetLastError();
}

hipError_t launch_col_detect(const float2* state, int nwaves, int n, const float2* prop_p,
                             const float2* twN, const DetBins& bins, double* partial,
                             hipStream_t st) {
#define COLD(NN)                                                                                 \
  hipLaunchKernelGGL((k_col_pass<NN, true>), dim3((unsigned)(nwaves * col_tiles(NN))),           \
                     dim3(col_nt(NN)), 0, st, const_cast<float2*>(state), prop_p, twN, bins,    \
                     partial)
  PRISM_DISPATCH_N(n, COLD)
#undef COLD
  return hipGetLastError();
}

hipError_t launch_probe_init(float2* state, const double* probe_xy, int p0, int np, int n,
                             const ProbeOptics& po, const int2* aper, const float2* twN,
                             hipStream_t st) {
#define PINIT(NN)                                                                                \
  hipLaunchKernelGGL(k_probe_init<NN>, dim3((unsigned)(np * col_tiles(NN))), dim3(col_nt(NN)), 0, \
                     st, state, probe_xy, p0, po, aper, twN)
  PRISM_DISPATCH_N(n, PINIT)
#undef PINIT
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int nwaves, int tiles, int n_det,
                                  double* out, OutAcc acc, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for((size_t)nwaves * n_det, 256)), dim3(256),
                     0, st, partial, nwaves, tiles, n_det, out, acc);
  return hipGetLastError();
}

hipError_t launch_extract(const float2* state, int nwaves, int n, float2* smatrix,
                          const float2* twH, hipStream_t st) {
#define EXT(NN)                                                                                  \
  hipLaunchKernelGGL(k_extract<NN>, dim3((unsigned)((size_t)nwaves * (NN / 2) / ext_nseq(NN))),  \
                     dim3(256), 0, st, state, smatrix, twH)
  PRISM_DISPATCH_N(n, EXT)
#undef EXT
  return hipGetLastError();
}

}  // namespace prism
