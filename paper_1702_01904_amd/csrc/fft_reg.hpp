// Register-resident DFTs of length 16, 32 and 64 for the four-step slice
// passes (Eq. 5 needs a forward and an inverse transform per slice).
//
// A length R = R1 * R2 transform with x = R2 a + b and k = c + R1 d is
//     X[c + R1 d] = sum_b w_R2^{bd} [ w_R^{bc} sum_a x[R2 a + b] w_R1^{ac} ]
// (w_L = exp(-+2 pi i / L)): R2 DFTs of length R1, a twiddle w_R^{bc} per
// element, R1 DFTs of length R2. Everything stays in one thread's
// registers; the inner twiddles are compile-time constants.
//
// Pruning comes from the callers: inputs known to be zero are passed as
// literal zeros (the device code is built with -fno-signed-zeros so that
// x + 0 folds), outputs that are not used are removed as dead code.
#pragma once

#include "fft_lds.hpp"

namespace prism {

// cos(2 pi m / 64) for m in [0, 16].
__host__ __device__ constexpr float cos64_q1(int m) {
  return m == 0    ? 1.0f
         : m == 1  ? 0.99518472667219692873f
         : m == 2  ? 0.98078528040323043058f
         : m == 3  ? 0.95694033573220882438f
         : m == 4  ? 0.92387953251128673848f
         : m == 5  ? 0.88192126434835504956f
         : m == 6  ? 0.83146961230254523567f
         : m == 7  ? 0.77301045336273699338f
         : m == 8  ? 0.70710678118654757274f
         : m == 9  ? 0.63439328416364548779f
         : m == 10 ? 0.55557023301960228867f
         : m == 11 ? 0.47139673682599780857f
         : m == 12 ? 0.38268343236508983729f
         : m == 13 ? 0.29028467725446233105f
         : m == 14 ? 0.19509032201612833135f
         : m == 15 ? 0.09801714032956077016f
                   : 0.0f;
}

// cos and sin of 2 pi m / 64 for any integer m, from the first quadrant.
__host__ __device__ constexpr float cos64(int m) {
  return (m & 63) <= 16   ? cos64_q1(m & 63)
         : (m & 63) <= 32 ? -cos64_q1(32 - (m & 63))
         : (m & 63) <= 48 ? -cos64_q1((m & 63) - 32)
                          : cos64_q1(64 - (m & 63));
}
__host__ __device__ constexpr float sin64(int m) { return cos64(m - 16); }

// a * exp(-+2 pi i m / R), forward sign for INV = false; R divides 64.
// m is a compile-time constant after unrolling, so the branches fold and
// quarter turns cost no arithmetic.
template <int R, bool INV>
__host__ __device__ __forceinline__ float2 rot(float2 a, int m) {
  const int q = (m * (64 / R)) & 63;
  if (q == 0) return a;
  if (q == 16) return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  if (q == 32) return make_float2(-a.x, -a.y);
  if (q == 48) return INV ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  const float c = cos64(q), s = INV ? sin64(q) : -sin64(q);
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// a + b w^m and a - b w^m (w = exp(-+2 pi i / R)) with the rotation folded
// into the sum: for |cos| >= |sin|, b w^m = cos (b.x - b.y tan, b.y + b.x tan)
// (else sin times the cotangent form), so each output component is one
// multiply-add of a prepared term instead of a product and a sum. m is a
// compile-time constant after unrolling; quarter turns cost no arithmetic.
template <int R, bool INV>
__host__ __device__ __forceinline__ void rot_pm(float2 a, float2 b, int m, float2& plus,
                                                float2& minus) {
  const int q = (m * (64 / R)) & 63;
  if (q % 16 == 0) {
    const float2 r = rot<R, INV>(b, m);
    plus = make_float2(a.x + r.x, a.y + r.y);
    minus = make_float2(a.x - r.x, a.y - r.y);
    return;
  }
  const float c = cos64(q), s = INV ? sin64(q) : -sin64(q);
  const bool cdom = (c < 0 ? -c : c) >= (s < 0 ? -s : s);
  const float k = cdom ? c : s;          // factored-out scale
  const float t = cdom ? s / c : c / s;  // tangent or cotangent
  // u = b w^m / k
  const float2 u = cdom ? make_float2(b.x - b.y * t, b.y + b.x * t)
                        : make_float2(b.x * t - b.y, b.y * t + b.x);
  plus = make_float2(a.x + k * u.x, a.y + k * u.y);
  minus = make_float2(a.x - k * u.x, a.y - k * u.y);
}

template <int R>
struct RegSplit {
  static constexpr int R2 = R <= 32 ? 4 : 8;  // inner transforms run over a (length R1)
  static constexpr int R1 = R / R2;
};

// In-place length-R DFT, natural order in and out, not normalised.
template <int R, bool INV>
__host__ __device__ __forceinline__ void dft_reg(float2 (&v)[R]) {
  if constexpr (R <= 8) {
    dft<R, INV>(v);
  } else {
    constexpr int R1 = RegSplit<R>::R1, R2 = RegSplit<R>::R2;
    float2 y[R2][R1];
#pragma unroll
    for (int b = 0; b < R2; ++b) {
#pragma unroll
      for (int a = 0; a < R1; ++a) y[b][a] = v[R2 * a + b];
      dft<R1, INV>(y[b]);
    }
    if constexpr (R2 == 4) {
      // length-4 DFTs over b with the twiddles w_R^{bc} folded into their
      // first butterflies (rot_pm)
#pragma unroll
      for (int c = 0; c < R1; ++c) {
        float2 t0, t1, t2, tm;
        rot_pm<R, INV>(y[0][c], y[2][c], 2 * c, t0, t1);
        rot_pm<R, INV>(rot<R, INV>(y[1][c], c), y[3][c], 3 * c, t2, tm);
        const float2 t3 = mul_mi<INV>(tm);
        v[c] = cadd(t0, t2);
        v[c + R1] = cadd(t1, t3);
        v[c + 2 * R1] = csub(t0, t2);
        v[c + 3 * R1] = csub(t1, t3);
      }
    } else {
#pragma unroll
      for (int b = 1; b < R2; ++b)
#pragma unroll
        for (int c = 1; c < R1; ++c) y[b][c] = rot<R, INV>(y[b][c], b * c);
#pragma unroll
      for (int c = 0; c < R1; ++c) {
        float2 z[R2];
#pragma unroll
        for (int b = 0; b < R2; ++b) z[b] = y[b][c];
        dft<R2, INV>(z);
#pragma unroll
        for (int d = 0; d < R2; ++d) v[c + R1 * d] = z[d];
      }
    }
  }
}

}  // namespace prism
