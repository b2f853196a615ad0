// K2 for the factored plans: apodization and the lateral DFT (Eq. 1, F_x) as an FFT whose
// last stage lands directly in the factored coefficient order.
//
// The sub-aperture's channel spectra u_i[l] = a_i[l] X_l sit on grid columns
// x_l = col0 + col_step l (zero elsewhere) and P_i(q) = sum_x v_i[x] e^{-2 pi i q x / N}.
// With N = 16 N2, x = 16 xa + xb and q = N2 q1 + r the kernel of the sum splits as
//     e^{-2 pi i r xa / N2} e^{-2 pi i r xb / N} e^{-2 pi i q1 xb / 16},
// so
//   stage A  Y(xb, r)  = sum_xa v[16 xa + xb] e^{-2 pi i r xa / N2}   (N2-point FFT per xb)
//   twiddle  Y'(xb, r) = Y(xb, r) e^{-2 pi i r xb / N}
//   stage B  P(N2 q1 + r) = sum_xb Y'(xb, r) e^{-2 pi i q1 xb / 16}  (16-point FFT per r)
// and stage B's sixteen outputs for one r are slots r 16 + q1, q1 = 0..15: the order K3's
// factored kernels stage (coefficient q = (N/16) q1 + r in row r).
//
// One wave per (frame, bin): lane (i, xb) runs stage A of sub-aperture i, lane (i, r) stage
// B, the two meeting in the wave's LDS block [i][r][xb].  The stage-B results go back to
// the same rows; the wave then takes the largest magnitude (for the FP16 power-of-two
// scale, as in k2_lateral) and writes the bin's n_sub N coefficients coalesced.  The
// transforms are radix-4 FFTs in registers (about 10 operations per point and stage,
// against 8 L per point for the direct sum).
#pragma once
#include "kernels.hpp"

namespace pam {

// times S i
template <int S>
__device__ __forceinline__ float2 mul_si(float2 a) {
  return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// in-register DFTs with kernel e^{S 2 pi i n k / R}, natural order in and out
template <int S>
__device__ __forceinline__ void dft4s(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), b0 = cadd(x1, x3), b1 = mul_si<S>(csub(x1, x3));
  x0 = cadd(a0, b0);
  x2 = csub(a0, b0);
  x1 = cadd(a1, b1);
  x3 = csub(a1, b1);
}
// 16 points at v[o], v[o + st], ..., v[o + 15 st]: n = 4 n1 + n2, k = k1 + 4 k2
template <int S, int ST = 1>
__device__ __forceinline__ void dft16s(float2* v) {
  constexpr float C1 = 0.92387953251128674f;   // cos(pi / 8)
  constexpr float S1 = 0.38268343236508977f;   // sin(pi / 8)
  constexpr float R2 = 0.70710678118654752f;   // cos(pi / 4)
  float2 T[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T[n2][0] = v[ST * n2];
    T[n2][1] = v[ST * (4 + n2)];
    T[n2][2] = v[ST * (8 + n2)];
    T[n2][3] = v[ST * (12 + n2)];
    dft4s<S>(T[n2][0], T[n2][1], T[n2][2], T[n2][3]);
  }
  // twiddles e^{S 2 pi i n2 k1 / 16}
  auto rot = [](float2 x, float c, float s) { return make_float2(x.x * c - x.y * s, x.x * s + x.y * c); };
  T[1][1] = rot(T[1][1], C1, S * S1);
  T[1][2] = rot(T[1][2], R2, S * R2);
  T[1][3] = rot(T[1][3], S1, S * C1);
  T[2][1] = rot(T[2][1], R2, S * R2);
  T[2][2] = mul_si<S>(T[2][2]);
  T[2][3] = rot(T[2][3], -R2, S * R2);
  T[3][1] = rot(T[3][1], S1, S * C1);
  T[3][2] = rot(T[3][2], -R2, S * R2);
  T[3][3] = rot(T[3][3], -C1, -S * S1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 y0 = T[0][k1], y1 = T[1][k1], y2 = T[2][k1], y3 = T[3][k1];
    dft4s<S>(y0, y1, y2, y3);
    v[ST * k1] = y0;
    v[ST * (k1 + 4)] = y1;
    v[ST * (k1 + 8)] = y2;
    v[ST * (k1 + 12)] = y3;
  }
}
// 8 points: n = 4 n1 + n2 (n1 < 2), k = k1 + 2 k2
template <int S>
__device__ __forceinline__ void dft8s(float2* v) {
  constexpr float R2 = 0.70710678118654752f;
  float2 T[4][2];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T[n2][0] = cadd(v[n2], v[4 + n2]);
    T[n2][1] = csub(v[n2], v[4 + n2]);
  }
  T[1][1] = make_float2(R2 * (T[1][1].x - S * T[1][1].y), R2 * (S * T[1][1].x + T[1][1].y));    // e^{S i pi / 4}
  T[2][1] = mul_si<S>(T[2][1]);                                                                    // S i
  T[3][1] = make_float2(-R2 * (T[3][1].x + S * T[3][1].y), R2 * (S * T[3][1].x - T[3][1].y));   // e^{S 3 i pi / 4}
#pragma unroll
  for (int k1 = 0; k1 < 2; ++k1) {
    float2 y0 = T[0][k1], y1 = T[1][k1], y2 = T[2][k1], y3 = T[3][k1];
    dft4s<S>(y0, y1, y2, y3);
    v[k1] = y0;
    v[k1 + 2] = y1;
    v[k1 + 4] = y2;
    v[k1 + 6] = y3;
  }
}
// 32 points: the 16-point transforms of the even and odd samples, then X[k] = E[k] + w^k O[k],
// X[k + 16] = E[k] - w^k O[k], w = e^{S 2 pi i / 32}
template <int S>
__device__ __forceinline__ void dft32s(float2* v) {
  // cos and sin of k pi / 16
  constexpr float CK[16] = {1.0f, 0.98078528040323043f, 0.92387953251128674f, 0.83146961230254524f,
                            0.70710678118654752f, 0.55557023301960229f, 0.38268343236508977f, 0.19509032201612833f,
                            0.0f, -0.19509032201612833f, -0.38268343236508977f, -0.55557023301960229f,
                            -0.70710678118654752f, -0.83146961230254524f, -0.92387953251128674f, -0.98078528040323043f};
  constexpr float SK[16] = {0.0f, 0.19509032201612833f, 0.38268343236508977f, 0.55557023301960229f,
                            0.70710678118654752f, 0.83146961230254524f, 0.92387953251128674f, 0.98078528040323043f,
                            1.0f, 0.98078528040323043f, 0.92387953251128674f, 0.83146961230254524f,
                            0.70710678118654752f, 0.55557023301960229f, 0.38268343236508977f, 0.19509032201612833f};
  dft16s<S, 2>(v);
  dft16s<S, 2>(v + 1);
  float2 out[32];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float2 t = cmul(make_float2(CK[k], S * SK[k]), v[2 * k + 1]);
    out[k] = cadd(v[2 * k], t);
    out[k + 16] = csub(v[2 * k], t);
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = out[k];
}
template <int S, int R>
__device__ __forceinline__ void dftn(float2* v) {
  if constexpr (R == 8) dft8s<S>(v);
  else if constexpr (R == 16) dft16s<S>(v);
  else dft32s<S>(v);
}

template <int NSUB, int N2>
__global__ __launch_bounds__(256) void k2_fft(K2Args a) {
  constexpr int N = 16 * N2;
  constexpr int RB = 17;                                     // padded row of 16 complex
  __shared__ float2 tr[4][NSUB][N2][RB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int item = blockIdx.x * 4 + w;                       // f n_sel + b
  if (item >= a.n_items) return;                             // wave-uniform; no workgroup barrier below
  const float2* X = a.spectra + (size_t)item * a.L;
  // stage A: lane (i, xb)
  if (lane < 16 * NSUB) {
    const int i = lane >> 4, xb = lane & 15;
    const float* mk = a.masks + i * a.L;
    float2 v[N2];
#pragma unroll
    for (int xa = 0; xa < N2; ++xa) {
      const int d = 16 * xa + xb - a.col0;                   // grid column minus the first element's
      const int l = a.col_step == 1 ? d : d / a.col_step;
      v[xa] = make_float2(0.f, 0.f);
      if (d >= 0 && d - l * a.col_step == 0 && l < a.L) {
        const float2 x = X[l];
        const float m = mk[l];
        v[xa] = make_float2(m * x.x, m * x.y);
      }
    }
    dftn<-1, N2>(v);
#pragma unroll
    for (int r = 0; r < N2; ++r) tr[w][i][r][xb] = cmul(v[r], a.twx[(r * xb) % N]);
  }
  __builtin_amdgcn_wave_barrier();
  // stage B: lane (i, r), 64 at a time; results back into the row, scaled by 1 / N
  const float invN = 1.0f / (float)N;
  float mx = 0.f;
  for (int it = lane; it < NSUB * N2; it += 64) {
    const int i = it / N2, r = it - (it / N2) * N2;
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = tr[w][i][r][k];
    dft16s<-1>(v);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      v[k] = make_float2(v[k].x * invN, v[k].y * invN);
      mx = fmaxf(mx, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
      tr[w][i][r][k] = v[k];
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  int ex = 0;
  frexpf(mx, &ex);                                           // mx = m 2^ex, m in [0.5, 1)
  const float scale = (a.scaled && mx > 0.f) ? ldexpf(1.0f, 12 - ex) : 1.0f;
  float2* dst = a.coeffs + (size_t)item * NSUB * N;
  for (int e = lane; e < NSUB * N; e += 64) {
    const int i = e / N, s = e - (e / N) * N;                // slot s = 16 r + q1
    const float2 c = tr[w][i][s >> 4][s & 15];
    dst[e] = make_float2(c.x * scale, c.y * scale);
  }
  if (lane == 0) a.inv_scale[item] = 1.0f / scale;
}

}  // namespace pam
