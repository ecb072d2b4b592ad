// PRISM window sum (Eq. PRISMfinal over the window of Eq. RegionBounds) on
// a packed, pixel-major copy of the active beams of S: with 16-bit (BF16 or
// FP16) operands for callers that accept their rounding, or with FP32
// operands. Accumulation is FP32 in both.
//
//  * Every active beam plane S_a is multiplied by an exact power of two
//    scale[a] that brings its largest component below 1, and alpha_a is
//    divided by the same factor, so the product is unchanged in exact
//    arithmetic and FP16 stays in range.
//  * S is packed once per call into a pixel-major 16-bit copy
//    s16[pixel][beam] = (Re, Im), beam rows padded to 64 entries, so that
//    one 32-beam K block of a pixel is 128 contiguous bytes.
//  * alpha is written by k_alpha16 directly in the real-ified MFMA A layout
//    (rows 2g: (Re, -Im), rows 2g+1: (Im, Re)) per probe group and K block.
//  * v_mfma_f32_16x16x32_{bf16,f16}: lane l holds A[l%16][8(l/16)+j],
//    B[8(l/16)+j][l%16] (j < 8) and D[4(l/16)+i][l%16] (i < 4).
//  * FP32: a K block is 16 beams (the same 128 bytes per row). Each lane
//    reads 16 bytes = 4 K' values and feeds four v_mfma_f32_16x16x4f32
//    steps; K' is visited as 4 (l/16) + 16 ks + s on both operands, a
//    permutation of the block's 32 real K' indices, so the sum is the same.
//    The scale is 1.
//  * Staging: 16-bit K blocks pass through registers into padded LDS rows,
//    two blocks ahead (these sums wait on operand fetch); FP32 K blocks go
//    straight from global memory into XOR-swizzled LDS rows
//    (global_load_lds_dwordx4), one block ahead, which frees the staging
//    registers for reading both K steps' operands before their products.
//  * The 1 / (W sqrt(B_A)) normalisation is applied in FP32 at the end.
#include "fft_lds.hpp"
#include "kernels.hpp"

namespace prism {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap_mod16(long long v, int m) {
  long long r = v % m;
  return (int)(r < 0 ? r + m : r);
}

template <Prec P>
__device__ __forceinline__ uint32_t pack16(float lo, float hi) {
  uint16_t a, b;
  if constexpr (P == Prec::kBF16) {
    a = __builtin_bit_cast(uint16_t, (__bf16)lo);
    b = __builtin_bit_cast(uint16_t, (__bf16)hi);
  } else {
    a = __builtin_bit_cast(uint16_t, (_Float16)lo);
    b = __builtin_bit_cast(uint16_t, (_Float16)hi);
  }
  return (uint32_t)a | ((uint32_t)b << 16);
}

// One 16-byte operand pair: one 16x16x32 MFMA (16-bit) or four 16x16x4
// steps (FP32).
template <Prec P>
__device__ __forceinline__ floatx4 mfma16(u32x4 a, u32x4 b, floatx4 c) {
  if constexpr (P == Prec::kF32) {
    const floatx4 af = __builtin_bit_cast(floatx4, a), bf = __builtin_bit_cast(floatx4, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(af.x, bf.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(af.y, bf.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(af.z, bf.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(af.w, bf.w, c, 0, 0, 0);
    return c;
  }
  if constexpr (P == Prec::kBF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  } else if constexpr (P == Prec::kFP16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, a),
                                                  __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// Largest |Re|, |Im| of each active plane: kScaleSplit blocks per plane
// (enough blocks to fill the GPU even for a few beams), then one thread per
// beam folds the partial maxima into the power-of-two scale.
__global__ __launch_bounds__(256) void k_s16_absmax(const float2* __restrict__ S,
                                                    const ActiveBeam* __restrict__ act, int ns,
                                                    float* __restrict__ partial) {
  const int a = blockIdx.x, part = blockIdx.y, tid = threadIdx.x;
  const size_t per = (size_t)ns * ns / kScaleSplit;  // complex values per block (even)
  const float4* pl = reinterpret_cast<const float4*>(S + (size_t)act[a].plane * ns * ns +
                                                     (size_t)part * per);
  float m = 0.f;
  for (size_t i = tid; i < per / 2; i += 256) {
    const float4 v = pl[i];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __shared__ float red[4];
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0)
    partial[(size_t)a * kScaleSplit + part] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_s16_scale(const float* __restrict__ partial, int n_act,
                                                   float* __restrict__ scale) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= n_act) return;
  float mm = 0.f;
  for (int k = 0; k < kScaleSplit; ++k) mm = fmaxf(mm, partial[(size_t)a * kScaleSplit + k]);
  float sc = 1.f;
  if (mm > 0.f) {
    int e;
    frexpf(mm, &e);  // mm = fr * 2^e with fr in [0.5, 1), so mm < 2^e
    sc = ldexpf(1.f, -e);
  }
  scale[a] = sc;
}

// FP32: 16 beams x 64 pixels per workgroup, transposed through LDS; a pixel
// row holds n_actp (re, im) float pairs, zero past the active beams.
__global__ __launch_bounds__(256) void k_s32_pack(const float2* __restrict__ S,
                                                  const ActiveBeam* __restrict__ act, int n_act,
                                                  int n_actp, int ns, float2* __restrict__ s32) {
  __shared__ float2 tile[64][17];
  const int tid = threadIdx.x;
  const size_t pix0 = (size_t)blockIdx.x * 64;
  const int a0 = blockIdx.y * 16;
  const size_t npix = (size_t)ns * ns;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    const int j = idx / 64, px = idx % 64;
    const int a = a0 + j;
    tile[px][j] = a < n_act ? S[(size_t)act[a].plane * npix + pix0 + px] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    const int px = idx / 16, j = idx % 16;
    s32[(pix0 + px) * n_actp + a0 + j] = tile[px][j];
  }
}

// 32 beams x 64 pixels per workgroup, transposed through LDS.
template <Prec P>
__global__ __launch_bounds__(256) void k_s16_pack(const float2* __restrict__ S,
                                                  const ActiveBeam* __restrict__ act, int n_act,
                                                  int n_actp, int ns, const float* __restrict__ scale,
                                                  uint32_t* __restrict__ s16) {
  __shared__ uint32_t tile[64][33];
  const int tid = threadIdx.x;
  const size_t pix0 = (size_t)blockIdx.x * 64;
  const int a0 = blockIdx.y * 32;
  const size_t npix = (size_t)ns * ns;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int idx = tid + 256 * i;
    const int j = idx / 64, px = idx % 64;
    const int a = a0 + j;
    uint32_t v = 0u;
    if (a < n_act) {
      const float2 z = S[(size_t)act[a].plane * npix + pix0 + px];
      const float sc = scale[a];
      v = pack16<P>(z.x * sc, z.y * sc);
    }
    tile[px][j] = v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int idx = tid + 256 * i;
    const int px = idx / 32, j = idx % 32;
    s16[(pix0 + px) * n_actp + a0 + j] = tile[px][j];
  }
}

// One thread per (probe group, K block, probe g, beam bl): the A' entries of
// alpha'' = exp(i phase) / scale[a] (scale 1 for FP32), zero outside the
// probe / beam range.
template <Prec P>
__global__ void k_alpha16(const double* __restrict__ probe_xy, int p0, int np,
                          const ActiveBeam* __restrict__ act, int n_act, int f, int ns, int w,
                          ProbeOptics po, const float* __restrict__ scale, int group, int nblk,
                          size_t total, uint32_t* __restrict__ a16, int2* __restrict__ origin) {
  constexpr int KB = prec_block_beams(P);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int bl = (int)(i % KB);
  const int g = (int)((i / KB) % group);
  const int blk = (int)((i / ((size_t)KB * group)) % nblk);
  const size_t grp = i / ((size_t)KB * group * nblk);
  const size_t p = grp * group + g;
  const int a = blk * KB + bl;
  float re = 0.f, im = 0.f;
  if (p < (size_t)np && a < n_act) {
    const double x0 = probe_xy[2 * (p0 + p)], y0 = probe_xy[2 * (p0 + p) + 1];
    if (a == 0) {
      const double dxs = po.cell / (double)ns;
      const int cx = wrap_mod16((long long)floor(x0 / dxs + 0.5), ns);
      const int cy = wrap_mod16((long long)floor(y0 / dxs + 0.5), ns);
      origin[p] = make_int2(wrap_mod16((long long)cx - w / 2, ns),
                            wrap_mod16((long long)cy - w / 2, ns));
    }
    const double kx = (double)act[a].m * f, ky = (double)act[a].n * f;
    const double dx = kx - po.ktx, dy = ky - po.kty;
    const double q2 = (dx * dx + dy * dy) * (po.dq * po.dq);
    double t = -(0.5 * po.lam * q2 * po.C1 + 0.25 * po.lam * po.lam * po.lam * q2 * q2 * po.C3) -
               (kx * (x0 - po.sx) + ky * (y0 - po.sy)) * po.dq;
    t -= floor(t);
    double s, c;
    sincospi(2.0 * t, &s, &c);
    const double inv = P == Prec::kF32 ? 1.0 : 1.0 / (double)scale[a];
    re = (float)(c * inv);
    im = (float)(s * inv);
  }
  const size_t base = (grp * nblk + blk) * (size_t)(2 * group) * (kC16KB);
  uint32_t* r0 = a16 + base + (size_t)(2 * g) * kC16KB;
  uint32_t* r1 = r0 + kC16KB;
  if constexpr (P == Prec::kF32) {
    // row 2g: (Re a, -Im a), row 2g+1: (Im a, Re a) as float pairs
    r0[2 * bl] = __builtin_bit_cast(uint32_t, re);
    r0[2 * bl + 1] = __builtin_bit_cast(uint32_t, -im);
    r1[2 * bl] = __builtin_bit_cast(uint32_t, im);
    r1[2 * bl + 1] = __builtin_bit_cast(uint32_t, re);
  } else {
    r0[bl] = pack16<P>(re, -im);
    r1[bl] = pack16<P>(im, re);
  }
}

// Workgroup shape per group size and operand form. Both shapes cover 128
// union pixels. FP32 (bound by the matrix cores) gives each of 4 waves two
// 16-pixel column tiles at two waves per SIMD; the 16-bit forms (bound by
// operand fetch) give each of 8 waves one tile at four waves per SIMD, so
// more waves cover each other's waits, for groups whose A block (2G rows of
// 8 16-byte segments) has at least one segment per thread (G >= 32).
template <int G, Prec P>
struct C16Shape {
  static constexpr bool kWide = P != Prec::kF32 && G >= 32;
  static constexpr int NT = kWide ? 512 : 256;  // threads per workgroup
  static constexpr int CT = kWide ? 1 : 2;      // 16-pixel column tiles per wave
  static constexpr int WPE = kWide ? 4 : 2;     // waves per SIMD (register budget)
};
constexpr int kTile16 = 128;  // union pixels per workgroup
constexpr int kPitch16 = 36;             // uint32 per LDS row (32 + 4 pad)

struct UnionGeom16 {
  int y0, x0, uy, ux;
};

template <int G, Prec P>
__device__ __forceinline__ void contract16_tile(const uint32_t* __restrict__ s16, int rowlen,
                                                const uint32_t* __restrict__ a16g, int np,
                                                int p_base, int gcount, int ns, int w,
                                                const UnionGeom16& U, int tile, const int* offx,
                                                const int* offy, const int* rylo,
                                                const int* ryhi, int only, float out_scale,
                                                uint32_t* __restrict__ smem, uint32_t* buf0,
                                                uint32_t* buf1, float2* __restrict__ window) {
  constexpr int kNT16 = C16Shape<G, P>::NT, kCT16 = C16Shape<G, P>::CT;
  static_assert(kNT16 / 64 * 16 * kCT16 == kTile16, "a workgroup covers one union tile");
  static_assert(2 * G * 8 % kNT16 == 0 && kTile16 * 8 % kNT16 == 0,
                "every thread stages whole 16-byte segments of A and B");
  constexpr int RT = G / 8;
  constexpr int AROWS = 2 * G;
  constexpr int ABUF = AROWS * kPitch16, BBUF = kTile16 * kPitch16;
  constexpr int NAQ = AROWS * 8 / kNT16;     // u32x4 of the A block per thread
  constexpr int NBQ = kTile16 * 8 / kNT16;   // u32x4 of the B block per thread
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int npix = U.uy * U.ux;
  const int nblk = rowlen / kC16KB;

  // Row tiles (8 probes each) this wave multiplies: those holding a probe
  // whose window meets a union row of the wave's 32 pixels. The skipped
  // products only reach outputs the epilogue never stores, so the stored
  // sums are the same. FP32 only: the 16-bit sums wait on operand fetch,
  // and the branches cost them more than the skipped products save.
  unsigned rmask = 0;
  if constexpr (P != Prec::kF32) {
    rmask = (1u << RT) - 1u;
  } else if (only >= 0) {
    rmask = 1u << (only / 8);
  } else {
    const int up0 = tile * kTile16 + 16 * kCT16 * wv;
    if (up0 < npix) {
      const int a0 = up0 / U.ux, a1 = (min(up0 + 16 * kCT16, npix) - 1) / U.ux;
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (rylo[r] <= a1 && ryhi[r] >= a0) rmask |= 1u << r;
    }
  }

  // S pixels this thread stages: tile column (tid + 256 i) / 8. Columns
  // past the union read pixel 0 instead; their outputs are never stored,
  // and a B column only reaches its own output column, so nothing needs
  // clearing. Rows of absent probes and beams are zero in the packed A.
  int spix[NBQ];
#pragma unroll
  for (int i = 0; i < NBQ; ++i) {
    const int up = tile * kTile16 + ((tid + kNT16 * i) >> 3);
    int off = 0;
    if (up < npix) {
      const int a = up / U.ux, b = up - a * U.ux;
      off = ((U.y0 + a) % ns) * ns + ((U.x0 + b) % ns);
    }
    spix[i] = off;
  }
  const uint32_t* s16q = s16 + 4 * (tid & 7);

  floatx4 acc[RT][kCT16];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < kCT16; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int krow = lane >> 4, mcol = lane & 15;

  if constexpr (P == Prec::kF32) {
    // Operands go from global memory straight into LDS
    // (global_load_lds_dwordx4: lane i of a wave's instruction writes its 16
    // bytes at the wave's LDS base + 16 i), one K block ahead of the
    // products, into two buffers that are separate LDS arrays (so the
    // compiler sees that reads of one never wait for loads into the other);
    // no registers stage them. An LDS row holds the 8 16-byte segments of
    // one A row or of one pixel's K block, segment s stored at s ^ (row & 7),
    // so the rows that one read instruction's lanes meet fall in different
    // banks.
    constexpr int P32 = kC16KB;  // LDS row: 32 words, no padding
    constexpr int AOFF = 0, BOFF = AROWS * P32;
    typedef __attribute__((address_space(3))) void* lds_ptr;
    auto issue = [&](uint32_t* buf, int blk) {
      const uint32_t* ab = a16g + (size_t)blk * AROWS * kC16KB;
#pragma unroll
      for (int i = 0; i < NAQ; ++i) {
        const int row = (tid + kNT16 * i) >> 3;
        const int seg = (tid & 7) ^ (row & 7);
        __builtin_amdgcn_global_load_lds(ab + (size_t)row * kC16KB + 4 * seg,
                                         (lds_ptr)(buf + AOFF + 4 * (kNT16 * i + 64 * wv)), 16, 0,
                                         0);
      }
#pragma unroll
      for (int i = 0; i < NBQ; ++i) {
        const int row = (tid + kNT16 * i) >> 3;
        const int seg = (tid & 7) ^ (row & 7);
        __builtin_amdgcn_global_load_lds(s16 + (size_t)spix[i] * rowlen + blk * kC16KB + 4 * seg,
                                         (lds_ptr)(buf + BOFF + 4 * (kNT16 * i + 64 * wv)), 16, 0,
                                         0);
      }
    };
    // both K steps' operands are read before the products, so the second
    // step's reads overlap the first step's products
    auto compute = [&](const uint32_t* buf) {
      const uint32_t* A = buf + AOFF + mcol * P32;
      const uint32_t* Bm = buf + BOFF + (16 * kCT16 * wv + mcol) * P32;
      u32x4 av[2][RT], bv[2][kCT16];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int seg = 4 * ((krow + 4 * ks) ^ (mcol & 7));
#pragma unroll
        for (int r = 0; r < RT; ++r)
          av[ks][r] = *reinterpret_cast<const u32x4*>(A + 16 * r * P32 + seg);
#pragma unroll
        for (int c = 0; c < kCT16; ++c)
          bv[ks][c] = *reinterpret_cast<const u32x4*>(Bm + 16 * c * P32 + seg);
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (rmask >> r & 1u)
#pragma unroll
            for (int c = 0; c < kCT16; ++c) acc[r][c] = mfma16<P>(av[ks][r], bv[ks][c], acc[r][c]);
    };
    // rows hold a whole number of K-block pairs: block 2j in buf0, 2j + 1
    // in buf1
    issue(buf0, 0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads are in LDS
    __syncthreads();
    for (int blk = 0; blk < nblk; blk += 2) {
      issue(buf1, blk + 1);
      compute(buf0);
      __builtin_amdgcn_s_waitcnt(0x0F70);
      // every wave's block blk + 1 is in LDS and no wave still reads buf0
      __syncthreads();
      if (blk + 2 < nblk) issue(buf0, blk + 2);
      compute(buf1);
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
    }
  } else {
    u32x4 ga[2][NAQ], gb[2][NBQ];
    auto fetch = [&](int set, int blk) {
      const u32x4* ab = reinterpret_cast<const u32x4*>(a16g + (size_t)blk * AROWS * kC16KB);
#pragma unroll
      for (int i = 0; i < NAQ; ++i) ga[set][i] = ab[tid + kNT16 * i];
#pragma unroll
      for (int i = 0; i < NBQ; ++i)
        gb[set][i] =
            *reinterpret_cast<const u32x4*>(s16q + (size_t)spix[i] * rowlen + blk * kC16KB);
    };
    auto stash = [&](int set) {
      uint32_t* A = smem + set * ABUF;
      uint32_t* Bm = smem + 2 * ABUF + set * BBUF;
#pragma unroll
      for (int i = 0; i < NAQ; ++i) {
        const int idx = tid + kNT16 * i;
        *reinterpret_cast<u32x4*>(A + (idx >> 3) * kPitch16 + 4 * (idx & 7)) = ga[set][i];
      }
#pragma unroll
      for (int i = 0; i < NBQ; ++i) {
        const int idx = tid + kNT16 * i;
        *reinterpret_cast<u32x4*>(Bm + (idx >> 3) * kPitch16 + 4 * (idx & 7)) = gb[set][i];
      }
    };
    auto compute = [&](int buf) {
      const uint32_t* A = smem + buf * ABUF + mcol * kPitch16 + 4 * krow;
      const uint32_t* Bm =
          smem + 2 * ABUF + buf * BBUF + (16 * kCT16 * wv + mcol) * kPitch16 + 4 * krow;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        u32x4 av[RT], bv[kCT16];
#pragma unroll
        for (int r = 0; r < RT; ++r)
          av[r] = *reinterpret_cast<const u32x4*>(A + 16 * r * kPitch16 + 16 * ks);
#pragma unroll
        for (int c = 0; c < kCT16; ++c)
          bv[c] = *reinterpret_cast<const u32x4*>(Bm + 16 * c * kPitch16 + 16 * ks);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int c = 0; c < kCT16; ++c) acc[r][c] = mfma16<P>(av[r], bv[c], acc[r][c]);
      }
    };

    // rows hold a whole number of K-block pairs
    fetch(0, 0);
    fetch(1, 1);
    for (int blk = 0; blk < nblk; blk += 2) {
      stash(0);
      __syncthreads();
      fetch(0, min(blk + 2, nblk - 2));
      compute(0);
      stash(1);
      __syncthreads();
      fetch(1, min(blk + 3, nblk - 1));
      compute(1);
    }
  }
  __syncthreads();

  const size_t w2 = (size_t)w * w;
#pragma unroll
  for (int c = 0; c < kCT16; ++c) {
    const int up = tile * kTile16 + 16 * kCT16 * wv + 16 * c + (lane & 15);
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
            make_float2(acc[r][c][2 * h] * out_scale, acc[r][c][2 * h + 1] * out_scale);
      }
    }
  }
}

// Grid: x walks the union tiles of a group, y the probe groups of every
// segment (segment k owns groups g_begin .. g_begin + ceil(np / G)).
template <int G, Prec P>
__global__ __launch_bounds__((C16Shape<G, P>::NT))
__attribute__((amdgpu_waves_per_eu(C16Shape<G, P>::WPE))) void k_contract16(
    const ContractSegs segs, int w) {
  // 16-bit operands: one array for both register-staged buffers; FP32: two
  // arrays, one per buffer (A block, then B block)
  constexpr bool F32 = P == Prec::kF32;
  constexpr int LDS = F32 ? 1 : 2 * (2 * G * kPitch16) + 2 * (kTile16 * kPitch16);
  constexpr int LDSB = F32 ? (2 * G + kTile16) * kC16KB : 1;
  __shared__ uint32_t smem[LDS];
  __shared__ uint32_t sbuf0[LDSB], sbuf1[LDSB];
  __shared__ int offx[G], offy[G];
  __shared__ int zero[G];
  __shared__ int ginfo[6];
  __shared__ int rylo[G / 8], ryhi[G / 8];  // union rows each row tile's windows span
  const int tid = threadIdx.x;
  int k = 0;  // segment of this group (uniform)
  while (k + 1 < segs.n && (int)blockIdx.y >= segs.s[k + 1].g_begin) ++k;
  const ContractSeg& sg = segs.s[k];
  const uint32_t* __restrict__ s16 = sg.s16;
  const int2* __restrict__ origin = sg.origin;
  const int rowlen = sg.rowlen, ns = sg.ns, np = sg.np;
  const int grp = (int)blockIdx.y - sg.g_begin;
  const int p_base = grp * G;
  const int gcount = min(G, np - p_base);
  const int nblk = rowlen / kC16KB;
  const uint32_t* a16g = sg.a16 + (size_t)grp * nblk * (2 * G) * kC16KB;
  if (tid < 64) {
    // group geometry in wave 0, one lane per probe (G <= 64): offsets of
    // each window from the first, their extent, and the union origin
    const int2 o0 = origin[p_base];
    int rx = 0, ry = 0;
    if (tid < gcount) {
      const int2 o = origin[p_base + tid];
      rx = wrap_mod16((long long)o.x - o0.x + ns / 2, ns) - ns / 2;
      ry = wrap_mod16((long long)o.y - o0.y + ns / 2, ns) - ns / 2;
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
      // one pass over the union of the windows costs (w + sx)(w + sy)
      // pixels, one pass per probe costs gcount w^2: take the cheaper (each
      // output pixel gets the same sum either way)
      const long long uni = (long long)(w + maxx - minx) * (w + maxy - miny);
      ginfo[0] = uni <= (long long)gcount * w * w ? 0 : 1;
      ginfo[1] = wrap_mod16((long long)o0.y + miny, ns);
      ginfo[2] = wrap_mod16((long long)o0.x + minx, ns);
      ginfo[3] = w + (maxy - miny);
      ginfo[4] = w + (maxx - minx);
    }
  }
  for (int g = tid; g < G; g += C16Shape<G, P>::NT) zero[g] = 0;
  __syncthreads();
  if (tid < G / 8) {
    int lo = 1 << 30, hi = -1;
    for (int j = 0; j < 8; ++j) {
      const int g = 8 * tid + j;
      if (g < gcount) {
        lo = min(lo, offy[g]);
        hi = max(hi, offy[g] + w - 1);
      }
    }
    rylo[tid] = lo;
    ryhi[tid] = hi;
  }
  __syncthreads();
  // the workgroups of a group share its tiles round-robin
  if (ginfo[0] == 0) {
    const UnionGeom16 U{ginfo[1], ginfo[2], ginfo[3], ginfo[4]};
    for (int tile = blockIdx.x; tile * kTile16 < U.uy * U.ux; tile += gridDim.x)
      contract16_tile<G, P>(s16, rowlen, a16g, np, p_base, gcount, ns, w, U, tile, offx, offy,
                            rylo, ryhi, -1, sg.out_scale, smem, sbuf0, sbuf1, sg.window);
  } else {
    for (int tile = blockIdx.x; tile * kTile16 < w * w; tile += gridDim.x) {
      for (int g = 0; g < gcount; ++g) {
        const int2 o = origin[p_base + g];
        const UnionGeom16 U{o.y, o.x, w, w};
        contract16_tile<G, P>(s16, rowlen, a16g, np, p_base, gcount, ns, w, U, tile, zero, zero,
                              rylo, ryhi, g, sg.out_scale, smem, sbuf0, sbuf1, sg.window);
      }
    }
  }
}

inline unsigned blocks16(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_s16_scale(const float2* smatrix, const ActiveBeam* act, int n_act, int ns,
                            float* partial, float* scale, hipStream_t st) {
  hipLaunchKernelGGL(k_s16_absmax, dim3((unsigned)n_act, (unsigned)kScaleSplit), dim3(256), 0, st,
                     smatrix, act, ns, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_s16_scale, dim3((unsigned)((n_act + 255) / 256)), dim3(256), 0, st, partial,
                     n_act, scale);
  return hipGetLastError();
}

hipError_t launch_s16_pack(const float2* smatrix, const ActiveBeam* act, int n_act, int n_actp,
                           int ns, const float* scale, void* s16, Prec prec, hipStream_t st) {
  const unsigned gx = (unsigned)((size_t)ns * ns / 64);
  if (prec == Prec::kF32) {
    hipLaunchKernelGGL(k_s32_pack, dim3(gx, (unsigned)(n_actp / 16)), dim3(256), 0, st, smatrix,
                       act, n_act, n_actp, ns, static_cast<float2*>(s16));
  } else if (prec == Prec::kBF16) {
    hipLaunchKernelGGL(k_s16_pack<Prec::kBF16>, dim3(gx, (unsigned)(n_actp / 32)), dim3(256), 0,
                       st, smatrix, act, n_act, n_actp, ns, scale, static_cast<uint32_t*>(s16));
  } else {
    hipLaunchKernelGGL(k_s16_pack<Prec::kFP16>, dim3(gx, (unsigned)(n_actp / 32)), dim3(256), 0,
                       st, smatrix, act, n_act, n_actp, ns, scale, static_cast<uint32_t*>(s16));
  }
  return hipGetLastError();
}

hipError_t launch_alpha16(const double* probe_xy, int p0, int np, const ActiveBeam* act,
                          int n_act, int n_actp, int f, int ns, int w, const ProbeOptics& po,
                          const float* scale, int group, void* a16, int2* origin, Prec prec,
                          hipStream_t st) {
  const int ngrp = (np + group - 1) / group;
  const int kb = prec_block_beams(prec);
  const int nblk = n_actp / kb;
  const size_t total = (size_t)ngrp * nblk * group * kb;
#define A16(PP)                                                                                \
  hipLaunchKernelGGL(k_alpha16<PP>, dim3(blocks16(total, 256)), dim3(256), 0, st, probe_xy, p0, \
                     np, act, n_act, f, ns, w, po, scale, group, nblk, total,                  \
                     static_cast<uint32_t*>(a16), origin)
  if (prec == Prec::kF32) A16(Prec::kF32);
  else if (prec == Prec::kBF16) A16(Prec::kBF16);
  else A16(Prec::kFP16);
#undef A16
  return hipGetLastError();
}

hipError_t launch_contract16(const ContractSegs& segs, int w, int group, Prec prec,
                             int window_tile_div, hipStream_t st) {
  if (segs.n < 1 || segs.n > kMaxSeg || segs.groups < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)contract_tile_slots(w, window_tile_div), (unsigned)segs.groups);
#define C16(GG, PP) \
  hipLaunchKernelGGL((k_contract16<GG, PP>), grid, dim3(C16Shape<GG, PP>::NT), 0, st, segs, w)
#define C16G(PP)                          \
  switch (group) {                        \
    case 16: C16(16, PP); break;          \
    case 32: C16(32, PP); break;          \
    case 64: C16(64, PP); break;          \
    default: return hipErrorInvalidValue; \
  }
  if (prec == Prec::kF32) {
    C16G(Prec::kF32)
  } else if (prec == Prec::kBF16) {
    C16G(Prec::kBF16)
  } else {
    C16G(Prec::kFP16)
  }
#undef C16G
#undef C16
  return hipGetLastError();
}

}  // namespace prism
