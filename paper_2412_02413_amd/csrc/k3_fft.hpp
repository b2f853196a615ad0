// K3 for FP32 operands at N = 128, 256 and 512: the inverse lateral transform as a 16 x N/16
// FFT on the vector ALUs.
//
// Same factorisation as k3_factored.hpp (q = (N/16) q1 + q2, x = x1 + 16 x2):
//   stage 1  Y(x1, q2)  = sum_q1 A((N/16) q1 + q2) e^{2 pi i q1 x1 / 16}
//   twiddle  Y'(x1, q2) = Y(x1, q2) e^{2 pi i q2 x1 / N}
//   stage 3  p(x1 + 16 x2) = sum_q2 Y'(x1, q2) e^{2 pi i q2 x2 / (N/16)}
// but each small transform is a radix-4 FFT held in one lane's registers instead of a
// DFT-GEMM on the matrix cores.  On gfx950 the FP32 matrix product runs at twice the
// vector FMA rate and does not overlap vector work, while the GEMM form executes 256 flops
// per complex output against about 11 vector operations per point and stage for the FFT,
// so for FP32 operands the vector FFT is the faster form.  (The 16-bit forms keep the
// matrix cores, whose rate is eight times higher and which overlap vector work.)
//
// N = 256.  A wave holds four depths, one per group of 16 lanes (g = lane / 16), and lane j
// of a group holds column q2 = j of stage 1 and column x1 = j of stage 3, i.e. its pixels
// are x = j + 16 x2, x2 = 0..15.  Per bin and sub-aperture:
//   A(16 m + j) = H G for m = 0..15 from the staged row j (K2's [q2][q1] order),
//   16-point FFT over m, twiddle, transpose through the group's LDS block (row x1),
//   16-point FFT over q2: the 16 fields of the lane's pixels.
// The fold into the per-pixel sums is that of k3ff.  A workgroup is 4 waves = 16 depths of
// one frame, staging each bin's coefficients and kz row in LDS (double-buffered, one
// barrier per bin) exactly as k3ff does, so the workspace layout and K2 are shared.
// With COH (n_sub = 1) the adjacent-pixel pair sums come from lanes j ^ 1 (column
// partner) and g ^ 1, i.e. lane ^ 16 (depth partner).
//
// N = 128.  A group holds two depths: in stage 1 lane j is (depth j / 8, column q2 = j % 8)
// and reads staged row q2 (8 rows), so the transpose block row x1 holds both depths' eight
// q2 values; in stage 3 lane j = x1 runs two 8-point FFTs, one per depth, and its 16
// pixels are (depth d, x = j + 16 x2) for d = 0, 1 and x2 = 0..7.  A wave holds eight
// depths and a workgroup 32.
//
// N = 512 splits the sum by the parity e of q as k3ff does:
// p(x) = P_0(x mod 256) + e^{2 pi i x / 512} P_1(x mod 256), P_e the 256-point transform of
// A(2 q' + e).  The lane groups of a wave become (depth, e) = (g / 2, g % 2), so a wave holds
// two depths and a workgroup eight.  Lane (g, j) takes its inputs from staged row 2 j + e
// (q = 32 m + 2 j + e, K2's order for N / 16 = 32 rows); after stage 3 the lanes g and g ^ 1
// (lane ^ 16) exchange P_0 and P_1 of their 16 columns x' = j + 16 x2, and group e forms
// pixel x' + 256 e as P_0 +- w P_1 with w = e^{2 pi i x' / 512} (a 16 x 16 table in LDS).
#pragma once
#include "k3_factored.hpp"

namespace pam {

constexpr int kFtWaves = 4;                    // waves per workgroup
constexpr int kFtTr = 16 * kFfRow;             // float2 per lane group's transpose block [16 x1][kFfRow]

// depths per workgroup: 32 (N = 128), 16 (256), 8 (512)
template <int NN>
__host__ __device__ constexpr int ft_depths() { return NN == 128 ? 32 : (NN == 256 ? 16 : 8); }

// LDS: staged bins [2][ff_stage_rows], stage twiddles [16 x1][16 j], (N = 512) combination
// twiddles [2 e][16 x2][16 j], transpose blocks [4 waves][4 groups][kFtTr].
template <int NN>
__host__ __device__ constexpr int ft_twiddles() { return NN == 512 ? 768 : 256; }
template <int NSUB, int NN = 256>
inline size_t k3fft_lds() {
  return (size_t)(2 * ff_stage_rows<NSUB, NN / 16>() + ft_twiddles<NN>() + kFtWaves * 4 * kFtTr) * sizeof(float2);
}

// The 16-byte pieces of a bin's staged inputs, 256 per pass (one per thread): one pass at
// N = 128 and 256 (N = 128 with three sub-apertures fills it exactly), two parts of two
// passes at N = 512.  Separate members (not an array) so that they stay in registers.
template <int NSUB, int NN>
struct FtPiece {
  typedef FfRows<NSUB, NN / 16> P;
  static constexpr int R = NN == 512 ? 2 : 1;
  uint4 v0, v1, v2, v3;
  int d0, d1, d2, d3;
  __device__ FtPiece(int tid) {
    d0 = P::where(tid);
    d1 = NN > 128 ? P::where(tid + 256) : -1;
    d2 = R > 1 ? P::where(tid + 512) : -1;
    d3 = R > 1 ? P::where(tid + 768) : -1;
  }
  // pieces 0, 1 (part 0) and, at N = 512, pieces 2, 3 (part 1): the kernel moves the two
  // parts at different points of a bin so that only two are in registers at a time
  __device__ __forceinline__ void load(const K3Args& a, int f, int b, int tid, int part) {
    if (part == 0) {
      if (d0 >= 0) v0 = P::fetch(a, f, b, tid);
      if (NN > 128 && d1 >= 0) v1 = P::fetch(a, f, b, tid + 256);
    } else if (R > 1) {
      if (d2 >= 0) v2 = P::fetch(a, f, b, tid + 512);
      if (d3 >= 0) v3 = P::fetch(a, f, b, tid + 768);
    }
  }
  __device__ __forceinline__ void store(float2* stage, int part) const {
    if (part == 0) {
      if (d0 >= 0) *reinterpret_cast<uint4*>(stage + d0) = v0;
      if (NN > 128 && d1 >= 0) *reinterpret_cast<uint4*>(stage + d1) = v1;
    } else if (R > 1) {
      if (d2 >= 0) *reinterpret_cast<uint4*>(stage + d2) = v2;
      if (d3 >= 0) *reinterpret_cast<uint4*>(stage + d3) = v3;
    }
  }
};

__device__ __forceinline__ float2 f2add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 f2sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 f2iadd(float2 a, float2 b) { return make_float2(a.x - b.y, a.y + b.x); }  // a + i b
__device__ __forceinline__ float2 f2isub(float2 a, float2 b) { return make_float2(a.x + b.y, a.y - b.x); }  // a - i b

// In-register inverse 16-point DFT, natural order in and out:
//   v[k] <- sum_n v[n] e^{+2 pi i n k / 16}.
// Radix 4 x 4 with n = 4 n1 + n2 and k = k1 + 4 k2: 4-point transforms over n1, then for
// each k1 the 4-point transform over n2 of y_n2 = W^(n2 k1) T[n2][k1], W = e^{2 pi i / 16}.
// The twiddled inputs of that second transform are written as y = c (x + i t x), c and t
// the cosine and tangent of the twiddle angle, so that the rotation costs two FMAs and its
// cosine folds into the butterfly's FMAs; y1 +- y3 = c1 (u1 +- (c3 / c1) u3) shares the
// factor c1.  A twiddled column then takes 22 operations instead of 28 (20 instead of 24 at
// k1 = 2).  Every tangent and cosine ratio used lies within [-2.42, 2.42].
__device__ __forceinline__ float2 tan_rot(float2 x, float t) {   // x + i t x
  return make_float2(fmaf(-t, x.y, x.x), fmaf(t, x.x, x.y));
}
// second-stage column with general twiddles W^k1, W^2k1, W^3k1 (k1 = 1 or 3):
// y0 = x0, yj = cj uj with uj = xj + i tj xj; r = c3 / c1
__device__ __forceinline__ void idft4_tw(float2& x0, float2& x1, float2& x2, float2& x3, float c1, float t1, float c2,
                                         float t2, float t3, float r) {
  const float2 u1 = tan_rot(x1, t1), u2 = tan_rot(x2, t2), u3 = tan_rot(x3, t3);
  const float2 a0 = make_float2(fmaf(c2, u2.x, x0.x), fmaf(c2, u2.y, x0.y));      // y0 + y2
  const float2 a1 = make_float2(fmaf(-c2, u2.x, x0.x), fmaf(-c2, u2.y, x0.y));    // y0 - y2
  const float2 v = make_float2(fmaf(r, u3.x, u1.x), fmaf(r, u3.y, u1.y));         // (y1 + y3) / c1
  const float2 w = make_float2(fmaf(-r, u3.x, u1.x), fmaf(-r, u3.y, u1.y));       // (y1 - y3) / c1
  x0 = make_float2(fmaf(c1, v.x, a0.x), fmaf(c1, v.y, a0.y));
  x2 = make_float2(fmaf(-c1, v.x, a0.x), fmaf(-c1, v.y, a0.y));
  x1 = make_float2(fmaf(-c1, w.y, a1.x), fmaf(c1, w.x, a1.y));                   // a1 + i (y1 - y3)
  x3 = make_float2(fmaf(c1, w.y, a1.x), fmaf(-c1, w.x, a1.y));                   // a1 - i (y1 - y3)
}
__device__ __forceinline__ void idft16(float2 (&v)[16]) {
  constexpr float C1 = 0.92387953251128674f;   // cos(pi / 8)
  constexpr float S1 = 0.38268343236508977f;   // sin(pi / 8) = cos(3 pi / 8)
  constexpr float R2 = 0.70710678118654752f;   // cos(pi / 4)
  constexpr float T1 = 0.41421356237309505f;   // tan(pi / 8)
  constexpr float T3 = 2.41421356237309505f;   // tan(3 pi / 8)
  float2 T[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    const float2 a0 = f2add(v[n2], v[8 + n2]), a1 = f2sub(v[n2], v[8 + n2]);
    const float2 b0 = f2add(v[4 + n2], v[12 + n2]), b1 = f2sub(v[4 + n2], v[12 + n2]);
    T[n2][0] = f2add(a0, b0);
    T[n2][2] = f2sub(a0, b0);
    T[n2][1] = f2iadd(a1, b1);
    T[n2][3] = f2isub(a1, b1);
  }
  // k1 = 0: no twiddles
  {
    const float2 a0 = f2add(T[0][0], T[2][0]), a1 = f2sub(T[0][0], T[2][0]);
    const float2 b0 = f2add(T[1][0], T[3][0]), b1 = f2sub(T[1][0], T[3][0]);
    v[0] = f2add(a0, b0);
    v[8] = f2sub(a0, b0);
    v[4] = f2iadd(a1, b1);
    v[12] = f2isub(a1, b1);
  }
  // k1 = 1: W^1 (pi / 8), W^2 (pi / 4), W^3 (3 pi / 8)
  idft4_tw(T[0][1], T[1][1], T[2][1], T[3][1], C1, T1, R2, 1.0f, T3, S1 / C1);
  v[1] = T[0][1];
  v[5] = T[1][1];
  v[9] = T[2][1];
  v[13] = T[3][1];
  // k1 = 2: W^2 (pi / 4), W^4 = i, W^6 (3 pi / 4); y1 +- y3 = R2 (u1 -+ u3)
  {
    const float2 x0 = T[0][2], x2 = T[2][2];
    const float2 a0 = make_float2(x0.x - x2.y, x0.y + x2.x);                   // y0 + i x2
    const float2 a1 = make_float2(x0.x + x2.y, x0.y - x2.x);                   // y0 - i x2
    const float2 u1 = make_float2(T[1][2].x - T[1][2].y, T[1][2].y + T[1][2].x);   // (1 + i) x1
    const float2 u3 = make_float2(T[3][2].x + T[3][2].y, T[3][2].y - T[3][2].x);   // (1 - i) x3 = -(-1 + i) x3
    const float2 s = f2sub(u1, u3), d = f2add(u1, u3);                          // (y1 + y3), (y1 - y3) over R2
    v[2] = make_float2(fmaf(R2, s.x, a0.x), fmaf(R2, s.y, a0.y));
    v[10] = make_float2(fmaf(-R2, s.x, a0.x), fmaf(-R2, s.y, a0.y));
    v[6] = make_float2(fmaf(-R2, d.y, a1.x), fmaf(R2, d.x, a1.y));
    v[14] = make_float2(fmaf(R2, d.y, a1.x), fmaf(-R2, d.x, a1.y));
  }
  // k1 = 3: W^3 (3 pi / 8), W^6 (3 pi / 4), W^9 (9 pi / 8)
  idft4_tw(T[0][3], T[1][3], T[2][3], T[3][3], S1, T3, -R2, -1.0f, T1, -C1 / S1);
  v[3] = T[0][3];
  v[7] = T[1][3];
  v[11] = T[2][3];
  v[15] = T[3][3];
}

// Two workgroups per CU (at most 256 VGPRs a lane).  At N = 512 with three sub-apertures
// this spills a few values per bin to scratch, which measures faster (about 1.4x) than one
// workgroup per CU without spills.
// In-register inverse 8-point DFT of v[o..o+7], natural order in and out:
//   v[o + k] <- sum_n v[o + n] e^{+2 pi i n k / 8}.
// n = 4 n1 + n2, k = k1 + 2 k2: 2-point transforms over n1, twiddles e^{2 pi i n2 k1 / 8},
// 4-point transforms over n2.
__device__ __forceinline__ void idft8(float2 (&v)[16], int o) {
  constexpr float R2 = 0.70710678118654752f;   // cos(pi / 4)
  float2 T[4][2];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T[n2][0] = f2add(v[o + n2], v[o + 4 + n2]);
    T[n2][1] = f2sub(v[o + n2], v[o + 4 + n2]);
  }
  T[1][1] = make_float2(R2 * (T[1][1].x - T[1][1].y), R2 * (T[1][1].x + T[1][1].y));     // W8^1
  T[2][1] = make_float2(-T[2][1].y, T[2][1].x);                                          // W8^2 = i
  T[3][1] = make_float2(-R2 * (T[3][1].x + T[3][1].y), R2 * (T[3][1].x - T[3][1].y));    // W8^3
#pragma unroll
  for (int k1 = 0; k1 < 2; ++k1) {
    const float2 a0 = f2add(T[0][k1], T[2][k1]), a1 = f2sub(T[0][k1], T[2][k1]);
    const float2 b0 = f2add(T[1][k1], T[3][k1]), b1 = f2sub(T[1][k1], T[3][k1]);
    v[o + k1] = f2add(a0, b0);
    v[o + k1 + 4] = f2sub(a0, b0);
    v[o + k1 + 2] = f2iadd(a1, b1);
    v[o + k1 + 6] = f2isub(a1, b1);
  }
}

template <int NSUB, bool COH = false, int NN = 256>
__global__ __launch_bounds__(256, 2) void k3fft(K3Args a0, K3Groups grp) {
  static_assert(!COH || (NSUB == 1 && NN == 256), "pair cross-spectra come with the full-aperture sums at N = 256");
  static_assert(NN == 128 || NN == 256 || NN == 512, "N = 128, 256 or 512");
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int N = NN;
  constexpr int R = NN == 512 ? 2 : 1;
  constexpr bool HALF = NN == 128;
  constexpr int ROWS = NN / 16;
  extern __shared__ float2 lds_ft[];
  float2* stage = lds_ft;                                          // [2][ff_stage_rows]
  float2* twl = lds_ft + 2 * ff_stage_rows<NSUB, ROWS>();          // [16 x1][16 j] (+ [2 e][16 x2][16 j])
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int e = R == 2 ? (g & 1) : 0;                              // parity of q (N = 512)
  float2* tr = twl + ft_twiddles<NN>() + (w * 4 + g) * kFtTr;     // this group's transpose block
  // staged row of this lane's stage-1 inputs
  const int srow = HALF ? (j & 7) : (R == 1 ? j : 2 * j + e);
  K3Args a = a0;
  const WgFF wg(a, wg_group(a, grp));
  const int f = wg.f;
  // first depth of the lane's pixels, and the depth of its stage-1 column
  const int depth = HALF ? wg.dt * ft_depths<NN>() + 8 * w + 2 * g
                         : (R == 1 ? wg.dt * ft_depths<NN>() + 4 * w + g : wg.dt * ft_depths<NN>() + 2 * w + (g >> 1));
  const int depth1 = HALF ? depth + (j >> 3) : depth;
  const double z = depth1 < a.n_z ? a.z[depth1] : 0.0;

  // stage-1 -> stage-3 twiddles e^{2 pi i q2 x1 / 256} and (N = 512) the combination twiddles
  // e^{2 pi i (j + 16 x2 + 256 e) / 512}, the e = 1 half the negated e = 0 half (FP32 tables built in FP64)
  for (int k = tid; k < ft_twiddles<NN>(); k += 256) {
    const float2 t = k < 256 ? a.ff_tw_vec[k] : a.ff_tw2_vec[(k - 256) & 255];
    twl[k] = k < 512 ? t : make_float2(-t.x, -t.y);
  }

  float accS[NSUB][16];
  float accC[NP > 0 ? NP : 1][16];
  float accG[COH ? 4 : 1][16];
#pragma unroll
  for (int x2 = 0; x2 < 16; ++x2) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[i][x2] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[p][x2] = 0.f;
#pragma unroll
    for (int q = 0; q < (COH ? 4 : 1); ++q) accG[q][x2] = 0.f;
  }

  FtPiece<NSUB, NN> pc(tid);
  if (wg.b_begin < wg.b_end) {
#pragma unroll
    for (int part = 0; part < R; ++part) {
      pc.load(a, f, wg.b_begin, tid, part);
      pc.store(stage, part);
    }
  }
  __syncthreads();
  for (int b = wg.b_begin; b < wg.b_end; ++b) {
    const bool more = b + 1 < wg.b_end;
    float2* nxt = stage + ((b + 1 - wg.b_begin) & 1) * ff_stage_rows<NSUB, ROWS>();   // free since the last barrier
    if (more) pc.load(a, f, b + 1, tid, 0);
    const float2* st = stage + ((b - wg.b_begin) & 1) * ff_stage_rows<NSUB, ROWS>();
    const double* kzr = reinterpret_cast<const double*>(st + NSUB * ROWS * kFfRow) + srow * kFfRow;
    // propagator at q = 16 m + j (N = 256) or 32 m + 2 j + e (N = 512) (Eq. 2): phase in FP64 reduced to [-1/2, 1/2] cycle,
    // hardware sin/cos; evanescent values replaced in a branch only lanes holding any take.
    // kz(q) = kz(N - q).  At N = 256, N - (16 m + j) = 16 (15 - m) + (16 - j): lane j's H[m] for m > 8 is lane
    // (16 - j)'s H[15 - m] (same depth), and lane 0's is its own H[16 - m].  At N = 512 the even-q rows (e = 0)
    // pair the same way, N - (32 m + 2 j) = 32 (15 - m) + 2 (16 - j), and in the odd-q rows
    // N - (32 m + 2 j + 1) = 32 (15 - m) + 2 (15 - j) + 1 pairs lane j with lane 15 - j, none with itself.  At
    // N = 128 (q = 8 m + q2, q2 = j % 8, one depth per 8 lanes) the partner of q2 is 8 - q2 in the same 8 lanes,
    // and q2 = 0 pairs with itself.  So a lane computes H[0..8] and takes the other seven from its partner lane.
    constexpr int MD = 9;   // values computed directly
    float2 H[16];
#pragma unroll
    for (int m = 0; m < MD; ++m) {
      const double ph = z * kzr[m];
      const float r = (float)(ph - rint(ph));
      H[m] = make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
    if (a.ev_bin[b]) {
#pragma unroll
      for (int m = 0; m < MD; ++m)
        if (kzr[m] < 0.0) H[m] = propagator(z, kzr[m], a.zero_evanescent);
    }
    {
      const bool self = (HALF ? (j & 7) : j) == 0 && e == 0;
#pragma unroll
      for (int m = MD; m < 16; ++m) {
        const float2 o =
            HALF     ? make_float2(lane_mirror8(H[15 - m].x), lane_mirror8(H[15 - m].y))
            : R == 2 ? make_float2(lane_mirror16_odd_rows15(H[15 - m].x), lane_mirror16_odd_rows15(H[15 - m].y))
                     : make_float2(lane_mirror16(H[15 - m].x), lane_mirror16(H[15 - m].y));
        H[m] = self ? H[16 - m] : o;
      }
    }
    float2 p[NSUB][16];
#pragma unroll
    for (int i = 0; i < NSUB; ++i) {
      const float4* gr = reinterpret_cast<const float4*>(st + (i * ROWS + srow) * kFfRow);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float4 gg = gr[k];
        p[i][2 * k] = cmul(H[2 * k], make_float2(gg.x, gg.y));
        p[i][2 * k + 1] = cmul(H[2 * k + 1], make_float2(gg.z, gg.w));
      }
    }
#pragma unroll
    for (int i = 0; i < NSUB; ++i) {
      idft16(p[i]);                                                // Y(x1, q2 = j), x1 = 0..15
#pragma unroll
      for (int x1 = 0; x1 < 16; ++x1)   // (the twiddle of x1 = 0 is exactly 1; skipped at N = 512 only,
                                        // where it shortens the spill, 76 -> 20 bytes a lane; at N = 128
                                        // and 256 the compiler's allocation then spills)
        tr[x1 * kFfRow + j] = (R == 2 && x1 == 0) ? p[i][0] : cmul(p[i][x1], twl[x1 * 16 + j]);
      __builtin_amdgcn_wave_barrier();
      const float4* yr = reinterpret_cast<const float4*>(tr + j * kFfRow);   // row x1 = j
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float4 yy = yr[k];
        p[i][2 * k] = make_float2(yy.x, yy.y);
        p[i][2 * k + 1] = make_float2(yy.z, yy.w);
      }
      __builtin_amdgcn_wave_barrier();
      if constexpr (HALF) {
        idft8(p[i], 0);                                            // depth + 0: p(j + 16 x2), x2 = 0..7
        idft8(p[i], 8);                                            // depth + 1
      } else {
        idft16(p[i]);                                              // p(j + 16 x2), x2 = 0..15
      }
      if constexpr (R == 2) {
        // p(x' + 256 e) = P_0(x') + w P_1(x'), x' = j + 16 x2, w = e^{2 pi i (x' + 256 e) / 512}: the even row of
        // each row pair (e = 0) holds P_0(x'), the odd row P_1(x'), and one row swap hands both to both rows
#pragma unroll
        for (int x2 = 0; x2 < 16; ++x2) {
          const float2 re = rows_even_odd(p[i][x2].x), im = rows_even_odd(p[i][x2].y);   // (P_0, P_1) parts
          const float2 w2 = twl[256 + 256 * e + x2 * 16 + j];
          p[i][x2] = make_float2(fmaf(w2.x, re.y, fmaf(-w2.y, im.y, re.x)), fmaf(w2.x, im.y, fmaf(w2.y, re.y, im.x)));
          // combined here: sunk to the fold, the two swapped halves would stay live instead of the result
          asm volatile("" : "+v"(p[i][x2].x), "+v"(p[i][x2].y));
        }
        // the next bin's second half once every transform is done (fewer values live through the transforms)
        if (i == NSUB - 1 && more) {
          pc.store(nxt, 0);
          pc.load(a, f, b + 1, tid, 1);
        }
      }
    }
    // fold: S_i = sum |p_i|^2, C_ij = sum Re(p_i conj p_j) (Eq. 4) over the bins
#pragma unroll
    for (int x2 = 0; x2 < 16; ++x2) {
#pragma unroll
      for (int i = 0; i < NSUB; ++i) accS[i][x2] = fmaf(p[i][x2].x, p[i][x2].x, fmaf(p[i][x2].y, p[i][x2].y, accS[i][x2]));
      if constexpr (NSUB == 3) {
        accC[0][x2] = fmaf(p[0][x2].x, p[1][x2].x, fmaf(p[0][x2].y, p[1][x2].y, accC[0][x2]));
        accC[1][x2] = fmaf(p[1][x2].x, p[2][x2].x, fmaf(p[1][x2].y, p[2][x2].y, accC[1][x2]));
        accC[2][x2] = fmaf(p[2][x2].x, p[0][x2].x, fmaf(p[2][x2].y, p[0][x2].y, accC[2][x2]));
      } else if constexpr (NSUB == 2) {
        accC[0][x2] = fmaf(p[0][x2].x, p[1][x2].x, fmaf(p[0][x2].y, p[1][x2].y, accC[0][x2]));
      }
      if constexpr (COH) {
        const float pr = p[0][x2].x, pi = p[0][x2].y;
        const float lr = lane_xor1(pr), li = lane_xor1(pi);
        const float zr = lane_xor16(pr), zi = lane_xor16(pi);
        accG[0][x2] = fmaf(pr, lr, fmaf(pi, li, accG[0][x2]));
        accG[1][x2] = fmaf(pi, lr, fmaf(-pr, li, accG[1][x2]));
        accG[2][x2] = fmaf(pr, zr, fmaf(pi, zi, accG[2][x2]));
        accG[3][x2] = fmaf(pi, zr, fmaf(-pr, zi, accG[3][x2]));
      }
    }
    if (more) pc.store(nxt, R - 1);
    __syncthreads();
  }
  constexpr int NA = COH ? 5 : AccCount<NSUB>::total;
  const size_t plane = (size_t)a.n_z * N;
  float* base = a.accum + ((size_t)wg.sp * a.F + f) * NA * plane;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    // pixel of register k: (depth + k / 8, j + 16 (k % 8)) at N = 128, (depth, j + 16 k + 256 e) otherwise
    const int d = HALF ? depth + (k >> 3) : depth;
    if (d >= a.n_z) continue;
    float* dst = base + (size_t)d * N + j + (HALF ? 16 * (k & 7) : 16 * k + 256 * e);
#pragma unroll
    for (int i = 0; i < NSUB; ++i) dst[i * plane] = accS[i][k];
#pragma unroll
    for (int q = 0; q < NP; ++q) dst[(NSUB + q) * plane] = accC[q][k];
    if constexpr (COH) {
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(1 + q) * plane] = accG[q][k];
    }
  }
}

}  // namespace pam
