// Frequency-domain delay-and-sum fields with the cross-spectra epilogue (FD-TEA-TAX).
//
// The paper's comparison beamformer in its frequency-domain form (Appendix, "PAM with
// DAX and TAX"): the monochromatic field at pixel r is the element spectra advanced by
// their travel times from r,
//     p_i(r, w) = sum_l a_i[l] X_l(w) exp(+i w tau_l(r)),   tau_l(r) = |r - r_l| / c,
// the Fourier transform of the delay-and-sum of Eq. 6 (unit distance weights).  The
// sums over w of |p_i|^2 and Re(p_i^* p_j) then give the NCC, TAX weight and image
// exactly as for the angular-spectrum fields (K4).
//
// One thread per pixel.  Bins run in chunks of TEA_BC: the chunk's element spectra
// are staged in LDS (read by every thread, broadcast), and for each element the
// thread forms its distance to the pixel in FP64, the phase k u (u = distance fs /
// (n_t c), cycles per bin index) in FP64 reduced to [-1/2, 1/2] cycle, and the
// hardware sine and cosine; the advanced spectrum is added to the field of every
// sub-aperture that holds the element (a per-element bit set, uniform over the
// workgroup).  After the chunk the fields are folded into the six per-pixel sums.
// No delay table is stored: an FP32 table would leave phase errors of ~2e-5 cycle at
// 8 MHz, and the FP64 distance costs a few instructions per element and chunk.
#pragma once
#include "kernels.hpp"

namespace pam {

constexpr int TEA_BC = 8;          // bins per chunk
constexpr int TEA_THREADS = 256;   // pixels per workgroup

struct TeaArgs {
  const float2* spectra;   // [F][n_sel][L] (K1)
  const int32_t* ksel;     // [n_sel] bin index k on the call's record-length grid
  const int32_t* subs;     // [L] bit i set if sub-aperture i holds element l
  const double* z;         // [n_z] depths
  float* accum;            // [n_split][F][n_acc][n_z][N]
  double x_first;          // lateral coordinate of grid column 0
  double dx;               // grid spacing
  double xl_first;         // lateral coordinate of element 0
  double pitch;            // element pitch
  double cyc;              // fs / (n_t c): phase cycles per bin index per metre of path
  int32_t L, N, n_z, n_sel, F, n_split, bins_per_split, n_ptile;
};

template <int NSUB>
__global__ __launch_bounds__(TEA_THREADS) void k3_tea(TeaArgs a) {
  constexpr int NP = AccCount<NSUB>::pairs;
  extern __shared__ float2 xs[];                  // [TEA_BC][L]
  __shared__ int ks[TEA_BC];
  int bid = blockIdx.x;
  const int sp = bid % a.n_split; bid /= a.n_split;
  const int pt = bid % a.n_ptile; bid /= a.n_ptile;
  const int f = bid;
  const int b_begin = sp * a.bins_per_split;
  const int b_end = min(a.n_sel, b_begin + a.bins_per_split);
  const int pix = pt * TEA_THREADS + threadIdx.x;
  const int npix = a.n_z * a.N;
  const bool live = pix < npix;
  const int d = live ? pix / a.N : 0, j = live ? pix - (pix / a.N) * a.N : 0;
  const double z = a.z[d];
  const double x = a.x_first + j * a.dx;

  float accS[NSUB], accC[NP > 0 ? NP : 1];
#pragma unroll
  for (int i = 0; i < NSUB; ++i) accS[i] = 0.f;
#pragma unroll
  for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[p] = 0.f;

  for (int b0 = b_begin; b0 < b_end; b0 += TEA_BC) {
    const int nb = min(TEA_BC, b_end - b0);
    __syncthreads();
    const float2* src = a.spectra + ((size_t)f * a.n_sel + b0) * a.L;
    for (int e = threadIdx.x; e < nb * a.L; e += TEA_THREADS) xs[e] = src[e];
    if ((int)threadIdx.x < nb) ks[threadIdx.x] = a.ksel[b0 + threadIdx.x];
    __syncthreads();
    float2 p[NSUB][TEA_BC];
#pragma unroll
    for (int i = 0; i < NSUB; ++i)
#pragma unroll
      for (int c = 0; c < TEA_BC; ++c) p[i][c] = make_float2(0.f, 0.f);
    for (int l = 0; l < a.L; ++l) {
      const int bits = __builtin_amdgcn_readfirstlane(a.subs[l]);
      if (bits == 0) continue;
      const double ddx = x - (a.xl_first + l * a.pitch);
      const double u = sqrt(ddx * ddx + z * z) * a.cyc;      // cycles per bin index
#pragma unroll
      for (int c = 0; c < TEA_BC; ++c) {
        if (c < nb) {
          const double ph = (double)ks[c] * u;
          const float r = (float)(ph - rint(ph));
          const float2 e = make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
          const float2 v = cmul(xs[c * a.L + l], e);
#pragma unroll
          for (int i = 0; i < NSUB; ++i)
            if (bits & (1 << i)) p[i][c] = cadd(p[i][c], v);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < TEA_BC; ++c) {
#pragma unroll
      for (int i = 0; i < NSUB; ++i) accS[i] = fmaf(p[i][c].x, p[i][c].x, fmaf(p[i][c].y, p[i][c].y, accS[i]));
      if constexpr (NSUB == 3) {
        accC[0] = fmaf(p[0][c].x, p[1][c].x, fmaf(p[0][c].y, p[1][c].y, accC[0]));
        accC[1] = fmaf(p[1][c].x, p[2][c].x, fmaf(p[1][c].y, p[2][c].y, accC[1]));
        accC[2] = fmaf(p[2][c].x, p[0][c].x, fmaf(p[2][c].y, p[0][c].y, accC[2]));
      } else if constexpr (NSUB == 2) {
        accC[0] = fmaf(p[0][c].x, p[1][c].x, fmaf(p[0][c].y, p[1][c].y, accC[0]));
      }
    }
  }
  if (!live) return;
  constexpr int NA = AccCount<NSUB>::total;
  const size_t plane = (size_t)npix;
  float* dst = a.accum + ((size_t)sp * a.F + f) * NA * plane + pix;
#pragma unroll
  for (int i = 0; i < NSUB; ++i) dst[i * plane] = accS[i];
#pragma unroll
  for (int q = 0; q < NP; ++q) dst[(NSUB + q) * plane] = accC[q];
}

}  // namespace pam
