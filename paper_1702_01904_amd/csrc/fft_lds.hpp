// LDS-resident batched FFTs for gfx950 (64-wide wavefronts).
//
// The multislice step (Eq. 5) needs a forward and an inverse 2D FFT per
// slice; the PRISM probe step (Fig. 1f) needs one small 2D FFT per probe.
// Both are done here as batches of 1D transforms held in LDS:
//   * Stockham auto-sort formulation, radix-8 stages followed by radix-4,
//     radix-2 and (for lengths 3 * 2^k and 9 * 2^k) radix-3 stages, so the
//     output is in natural order with no digit-reversal pass;
//   * each stage reads every butterfly input into registers, barriers,
//     then writes the outputs in place (one barrier pair per stage);
//   * twiddles come from a per-length table of exp(-2 pi i k / L), rounded
//     once from FP64, staged in LDS by the caller (the register DFTs of 3,
//     6, 9, 12 and 18 points use constants of cos(2 pi m / 36));
//   * LDS addresses are padded by one complex every 16 (lpad) to spread
//     the strided writes of early stages over the banks.
//
// A batch is described by compile-time strides: element e of sequence s is
// at flat index (s / SPB) * BSTR + (s % SPB) * SSTR + e * ESTR (before
// padding). SEQ_FAST picks whether consecutive threads walk sequences
// (strided sequences, e.g. columns) or elements (contiguous sequences).
// Forward transforms use exp(-2 pi i ...), inverse ones exp(+2 pi i ...);
// neither is normalised.
#pragma once

#include <hip/hip_runtime.h>

namespace prism {

constexpr int kPadShift = 4;

__host__ __device__ constexpr int lds_padded(int n) { return n + (n >> kPadShift); }
__device__ __forceinline__ int lpad(int i) { return i + (i >> kPadShift); }

__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft2(float2 (&v)[2]) {
  const float2 t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft4v(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft4(float2 (&v)[4]) {
  dft4v<INV>(v[0], v[1], v[2], v[3]);
}

// 8-point DFT as two 4-point DFTs (even/odd inputs) and a twiddled merge.
template <bool INV>
__host__ __device__ __forceinline__ void dft8(float2 (&v)[8]) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4v<INV>(e0, e1, e2, e3);
  dft4v<INV>(o0, o1, o2, o3);
  const float r = 0.70710678118654752440f;
  // o1 *= w^1, o2 *= w^2, o3 *= w^3 with w = exp(-+ 2 pi i / 8)
  if (INV) {
    o1 = make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y));
    o3 = make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y));
  } else {
    o1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
    o3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  }
  o2 = mul_mi<INV>(o2);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// 3-point DFT: X1, X2 = a - (b + c)/2 -+ i (sqrt(3)/2)(b - c) (forward).
template <bool INV>
__host__ __device__ __forceinline__ void dft3v(float2& a, float2& b, float2& c) {
  constexpr float h = 0.86602540378443864676f;  // sqrt(3) / 2
  const float2 t1 = cadd(b, c), t2 = csub(b, c);
  const float2 m = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
  const float2 r = mul_mi<INV>(make_float2(h * t2.x, h * t2.y));  // -+ i h (b - c)
  a = cadd(a, t1);
  b = cadd(m, r);
  c = csub(m, r);
}

template <bool INV>
__host__ __device__ __forceinline__ void dft3(float2 (&v)[3]) {
  dft3v<INV>(v[0], v[1], v[2]);
}

// cos and sin of 2 pi m / 12 for any integer m.
__host__ __device__ constexpr float cos12(int m) {
  return (m % 12 + 12) % 12 == 0    ? 1.0f
         : (m % 12 + 12) % 12 == 1  ? 0.86602540378443864676f
         : (m % 12 + 12) % 12 == 2  ? 0.5f
         : (m % 12 + 12) % 12 == 3  ? 0.0f
         : (m % 12 + 12) % 12 == 4  ? -0.5f
         : (m % 12 + 12) % 12 == 5  ? -0.86602540378443864676f
         : (m % 12 + 12) % 12 == 6  ? -1.0f
         : (m % 12 + 12) % 12 == 7  ? -0.86602540378443864676f
         : (m % 12 + 12) % 12 == 8  ? -0.5f
         : (m % 12 + 12) % 12 == 9  ? 0.0f
         : (m % 12 + 12) % 12 == 10 ? 0.5f
                                    : 0.86602540378443864676f;
}
__host__ __device__ constexpr float sin12(int m) { return cos12(m - 3); }

// a * exp(-+2 pi i m / 12) (forward sign for INV = false), m a compile-time
// constant after unrolling.
template <bool INV>
__host__ __device__ __forceinline__ float2 rot12(float2 a, int m) {
  const int q = (m % 12 + 12) % 12;
  if (q == 0) return a;
  if (q == 6) return make_float2(-a.x, -a.y);
  if (q == 3) return mul_mi<INV>(a);
  if (q == 9) return mul_mi<!INV>(a);
  const float c = cos12(q), s = INV ? sin12(q) : -sin12(q);
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// cos(2 pi m / 36) for m in [0, 9], and cos / sin of 2 pi m / 36 for any m.
__host__ __device__ constexpr float cos36_q1(int m) {
  return m == 0 ? 1.0f
         : m == 1 ? 0.98480775301220802032f
         : m == 2 ? 0.93969262078590842791f
         : m == 3 ? 0.86602540378443870761f
         : m == 4 ? 0.76604444311897801345f
         : m == 5 ? 0.64278760968653936292f
         : m == 6 ? 0.50000000000000011102f
         : m == 7 ? 0.34202014332566882393f
         : m == 8 ? 0.17364817766693041445f
         : m == 9 ? 0.00000000000000006123f
                : 0.0f;
}
__host__ __device__ constexpr float cos36(int m) {
  return (m % 36 + 36) % 36 <= 9    ? cos36_q1((m % 36 + 36) % 36)
         : (m % 36 + 36) % 36 <= 18 ? -cos36_q1(18 - (m % 36 + 36) % 36)
         : (m % 36 + 36) % 36 <= 27 ? -cos36_q1((m % 36 + 36) % 36 - 18)
                                    : cos36_q1(36 - (m % 36 + 36) % 36);
}
__host__ __device__ constexpr float sin36(int m) { return cos36(m - 9); }

// a * exp(-+2 pi i m / 36), m a compile-time constant after unrolling.
template <bool INV>
__host__ __device__ __forceinline__ float2 rot36(float2 a, int m) {
  const int q = (m % 36 + 36) % 36;
  if (q == 0) return a;
  if (q == 18) return make_float2(-a.x, -a.y);
  if (q == 9) return mul_mi<INV>(a);
  if (q == 27) return mul_mi<!INV>(a);
  const float c = cos36(q), s = INV ? sin36(q) : -sin36(q);
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// 9-point DFT as 3 x 3 and 18-point as 2 x 9 (Cooley-Tukey, x = R2 a + b).
template <int R1, int R2, bool INV>
__host__ __device__ __forceinline__ void dft_ct36(float2 (&v)[R1 * R2]) {
  constexpr int R = R1 * R2;
  float2 y[R2][R1];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
#pragma unroll
    for (int a = 0; a < R1; ++a) y[b][a] = v[R2 * a + b];
    if constexpr (R1 == 2) dft2<INV>(y[b]);
    else dft3<INV>(y[b]);
#pragma unroll
    for (int c = 1; c < R1; ++c) y[b][c] = rot36<INV>(y[b][c], (36 / R) * b * c);
  }
#pragma unroll
  for (int c = 0; c < R1; ++c) {
    float2 z[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) z[b] = y[b][c];
    if constexpr (R2 == 3) dft3<INV>(z);
    else dft_ct36<3, 3, INV>(z);
#pragma unroll
    for (int d = 0; d < R2; ++d) v[c + R1 * d] = z[d];
  }
}

// R = R1 * R2 (6 = 2 * 3, 12 = 4 * 3): R2 DFTs of length R1 over a
// (x = R2 a + b), twiddles w_R^{bc}, R1 DFTs of length R2 over b.
template <int R1, int R2, bool INV>
__host__ __device__ __forceinline__ void dft_ct12(float2 (&v)[R1 * R2]) {
  constexpr int R = R1 * R2;
  float2 y[R2][R1];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
#pragma unroll
    for (int a = 0; a < R1; ++a) y[b][a] = v[R2 * a + b];
    if constexpr (R1 == 2) dft2<INV>(y[b]);
    else dft4<INV>(y[b]);
#pragma unroll
    for (int c = 1; c < R1; ++c) y[b][c] = rot12<INV>(y[b][c], (12 / R) * b * c);
  }
#pragma unroll
  for (int c = 0; c < R1; ++c) {
    float2 z[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) z[b] = y[b][c];
    dft3<INV>(z);
#pragma unroll
    for (int d = 0; d < R2; ++d) v[c + R1 * d] = z[d];
  }
}

template <int R, bool INV>
__host__ __device__ __forceinline__ void dft(float2 (&v)[R]) {
  static_assert(R == 2 || R == 3 || R == 4 || R == 6 || R == 8 || R == 9 || R == 12 || R == 18,
                "register DFT lengths 2, 3, 4, 6, 8, 9, 12, 18");
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 6) dft_ct12<2, 3, INV>(v);
  else if constexpr (R == 12) dft_ct12<4, 3, INV>(v);
  else if constexpr (R == 9) dft_ct36<3, 3, INV>(v);
  else if constexpr (R == 18) dft_ct36<2, 9, INV>(v);
  else dft8<INV>(v);
}

// Batch geometry of LDS-held sequences (see header comment).
template <int L_, int NSEQ_, int SPB_, int BSTR_, int SSTR_, int ESTR_, bool SEQ_FAST_>
struct Batch {
  static constexpr int L = L_;
  static constexpr int NSEQ = NSEQ_;
  static constexpr int SPB = SPB_;
  static constexpr int BSTR = BSTR_;
  static constexpr int SSTR = SSTR_;
  static constexpr int ESTR = ESTR_;
  static constexpr bool SEQ_FAST = SEQ_FAST_;
  __device__ __forceinline__ static int addr(int s, int e) {
    return (s / SPB) * BSTR + (s % SPB) * SSTR + e * ESTR;
  }
};

// Contiguous sequences [NSEQ][L].
template <int L, int NSEQ>
using RowBatch = Batch<L, NSEQ, NSEQ, 0, L, 1, false>;

// Butterfly numbering of a stage: butterfly b -> (sequence s, index j).
template <class B, int NB>
__device__ __forceinline__ void stage_coords(int b, int& s, int& j) {
  if constexpr (B::SEQ_FAST) {
    s = b % B::NSEQ;
    j = b / B::NSEQ;
  } else {
    j = b % NB;
    s = b / NB;
  }
}

// Stockham stage of radix R with current span NS (product of the radices
// already applied), split into its two halves so that callers can keep a
// stage's inputs or outputs in registers:
//   stage_in  reads the R inputs of each butterfly of this thread from LDS
//             and applies the twiddles (none when NS == 1);
//   stage_out applies the R-point DFTs and writes the outputs to LDS.
// Butterfly j of sequence s reads elements j + r L/R and writes elements
// (j - k) R + k + r NS with k = j mod NS. tw: exp(-2 pi i m / L), m < L.
template <class B, int R, int NT>
struct StageShape {
  static constexpr int NB = B::L / R;
  static constexpr int TOT = B::NSEQ * NB;
  static constexpr int PER = (TOT + NT - 1) / NT;
  static constexpr bool GUARD = (TOT % NT) != 0;
};

// Padded address of flat index base + r * step: when step is a multiple of
// the padding period the pad term is r * step / 16, a compile-time offset.
template <int STEP>
__device__ __forceinline__ int lpad_step(int base_padded, int base, int r) {
  if constexpr (STEP % (1 << kPadShift) == 0) {
    return base_padded + r * (STEP + (STEP >> kPadShift));
  } else {
    return lpad(base + r * STEP);
  }
}

template <class B, int R, int NS, int NT, bool INV>
__device__ __forceinline__ void stage_in(const float2* lds, const float2* tw, int tid,
                                         float2 (&v)[StageShape<B, R, NT>::PER][R]) {
  using SS = StageShape<B, R, NT>;
  constexpr int TWS = B::L / (NS * R);
  constexpr int STEP = SS::NB * B::ESTR;
#pragma unroll
  for (int p = 0; p < SS::PER; ++p) {
    const int b = tid + p * NT;
    if (!SS::GUARD || b < SS::TOT) {
      int s, j;
      stage_coords<B, SS::NB>(b, s, j);
      const int k = j % NS;
      const int base = B::addr(s, j);
      const int pbase = lpad(base);
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = lds[lpad_step<STEP>(pbase, base, r)];
      if constexpr (NS > 1) {
        // twiddles w^r, w = exp(-+2 pi i k / (NS R)): w, w^2, w^4 from the
        // table, the other powers as products. The row pass is bound by LDS
        // traffic; this trades 4 of 7 table reads for complex products (the
        // FP32 path's error roughly doubles, ~1.7e-5 relative at 1024^2 and
        // 50 slices).
        float2 w[R];
        if constexpr (R == 2 || R == 4 || R == 8) {
          w[1] = tw[k * TWS];
          if constexpr (R >= 4) w[2] = tw[2 * k * TWS];
          if constexpr (R == 4) w[3] = cmul(w[1], w[2]);
          if constexpr (R == 8) {
            w[4] = tw[4 * k * TWS];
            w[3] = cmul(w[1], w[2]);
            w[5] = cmul(w[1], w[4]);
            w[6] = cmul(w[2], w[4]);
            w[7] = cmul(w[3], w[4]);
          }
        } else {  // radix 3, 6, 9, 12, 18: every power from the table
#pragma unroll
          for (int r = 1; r < R; ++r) w[r] = tw[r * k * TWS];
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = INV ? cmulc(v[p][r], w[r]) : cmul(v[p][r], w[r]);
      }
    }
  }
}

template <class B, int R, int NS, int NT, bool INV>
__device__ __forceinline__ void stage_out(float2* lds, int tid,
                                          float2 (&v)[StageShape<B, R, NT>::PER][R]) {
  using SS = StageShape<B, R, NT>;
#pragma unroll
  for (int p = 0; p < SS::PER; ++p) {
    const int b = tid + p * NT;
    if (!SS::GUARD || b < SS::TOT) {
      int s, j;
      stage_coords<B, SS::NB>(b, s, j);
      dft<R, INV>(v[p]);
      const int k = j % NS;
      const int o = (j - k) * R + k;
      constexpr int STEP = NS * B::ESTR;
      const int base = B::addr(s, o);
      const int pbase = lpad(base);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lpad_step<STEP>(pbase, base, r)] = v[p][r];
    }
  }
}

// One complete in-place stage (read, barrier, write, barrier).
template <class B, int R, int NS, int NT, bool INV>
__device__ __forceinline__ void fft_stage(float2* lds, const float2* tw, int tid) {
  float2 v[StageShape<B, R, NT>::PER][R];
  stage_in<B, R, NS, NT, INV>(lds, tw, tid, v);
  __syncthreads();
  stage_out<B, R, NS, NT, INV>(lds, tid, v);
  __syncthreads();
}

// COUNT consecutive radix-8 stages starting at span NS.
template <class B, int NT, bool INV, int NS, int COUNT>
__device__ __forceinline__ void fft_radix8_run(float2* lds, const float2* tw, int tid) {
  if constexpr (COUNT > 0) {
    fft_stage<B, 8, NS, NT, INV>(lds, tw, tid);
    fft_radix8_run<B, NT, INV, NS * 8, COUNT - 1>(lds, tw, tid);
  }
}

// Lengths handled by the LDS transforms: 2^k, 3 * 2^k or 9 * 2^k.
__host__ __device__ constexpr bool pow2_len(int L) { return L > 0 && (1 << ilog2(L)) == L; }
__host__ __device__ constexpr bool fft_len_ok(int L) {
  return pow2_len(L) || (L % 3 == 0 && pow2_len(L / 3)) || (L % 9 == 0 && pow2_len(L / 9));
}

// Radix plan of a length-L transform split as 8 * 8^MID * RL (RL in 2, 4, 8
// for L = 2^k; 3, 6, 12 for L = 3 * 2^k; 9, 18 for L = 9 * 2^k up to 1152):
// the inverse runs 8, 8^MID, RL and
// the forward the reverse RL, 8^MID, 8, so that the inverse's last stage
// and the forward's first stage pair up on the same elements (j + r L/RL)
// and can stay in registers.
template <int L>
struct PairedPlan {
  static constexpr int T = L % 9 == 0 ? 9 : (L % 3 == 0 ? 3 : 1);  // odd factor
  static constexpr int K = ilog2(L / T);
  // RL = T * 2^((K - 3) mod 3) for T > 1 (3, 6, 12 or 9, 18, 36)
  static constexpr int RL = T > 1 ? T * (1 << ((K - 3) % 3))
                                  : ((K % 3 == 1) ? 2 : ((K % 3 == 2) ? 4 : 8));
  static constexpr int MID = (K - 3 - ilog2(RL / T)) / 3;
};

template <class B, int NT, bool INV, int NS>
__device__ __forceinline__ void fft_from(float2* lds, const float2* tw, int tid) {
  constexpr int REM = B::L / NS;  // product of the radices still to apply
  if constexpr (REM % 8 == 0) {
    fft_stage<B, 8, NS, NT, INV>(lds, tw, tid);
    fft_from<B, NT, INV, NS * 8>(lds, tw, tid);
  } else if constexpr (REM % 4 == 0) {
    fft_stage<B, 4, NS, NT, INV>(lds, tw, tid);
    fft_from<B, NT, INV, NS * 4>(lds, tw, tid);
  } else if constexpr (REM % 2 == 0) {
    fft_stage<B, 2, NS, NT, INV>(lds, tw, tid);
    fft_from<B, NT, INV, NS * 2>(lds, tw, tid);
  } else if constexpr (REM % 3 == 0) {
    fft_stage<B, 3, NS, NT, INV>(lds, tw, tid);
    fft_from<B, NT, INV, NS * 3>(lds, tw, tid);
  }
}

// Full length-L transform of every sequence in the batch. The caller must
// have synchronised after writing the data and the twiddle table; on
// return the result is in LDS and visible to all threads.
template <class B, int NT, bool INV>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* tw, int tid) {
  static_assert(fft_len_ok(B::L), "lengths 2^k, 3 * 2^k or 9 * 2^k only");
  fft_from<B, NT, INV, 1>(lds, tw, tid);
}

// Copy a twiddle table from global memory into LDS (no barrier).
template <int L, int NT>
__device__ __forceinline__ void load_twiddles(float2* tw_lds, const float2* __restrict__ tw, int tid) {
  for (int i = tid; i < L; i += NT) tw_lds[i] = tw[i];
}

// Wavefront sum of a double (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace prism
