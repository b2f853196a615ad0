// K3 with the inverse lateral transform factored into two matrix-core DFT stages.
//
// The fields of one (frame, bin, depth) are p_i(x) = sum_q A_i(q) e^{+2 pi i q x / N},
// A_i(q) = H(q, z) G_i(q), with G_i the sub-aperture's lateral spectrum already
// divided by N (K2) and H the propagator of Eq. 2.  With N = N1 N2, q = N2 q1 + q2 and
// x = x1 + N1 x2 the kernel of the sum splits as
//     e^{2 pi i q1 x1 / N1} e^{2 pi i q2 x1 / N} e^{2 pi i q2 x2 / N2},
// so the transform is
//   stage 1  Y(x1, q2)  = sum_q1 A(N2 q1 + q2) e^{2 pi i q1 x1 / N1}   (N1-point DFTs)
//   twiddle  Y'(x1, q2) = Y(x1, q2) e^{2 pi i q2 x1 / N}
//   stage 3  p(x1 + N1 x2) = sum_q2 Y'(x1, q2) e^{2 pi i q2 x2 / N2}  (N2-point DFTs)
// Both DFT stages are complex GEMMs on the matrix cores against a constant 16-point
// DFT matrix in real form: rows (output index, re/im) = 32, K = (input index, re/im)
// = 32, and 32 independent transforms as the columns of one 32x32 tile.  Executed
// matrix flops per complex output are 2 x 128 instead of the 4N of a dense DFT.
//
// This file serves N = 256 (N1 = N2 = 16, R = 1) and N = 512 (R = 2).  At N = 256 a
// wave owns two depths and the full 256 columns: its stage-1 tile has columns
// (q2, depth) = 16 x 2, its stage-3 tile columns (x1, depth) = 16 x 2.  Between the
// stages each wave transposes its own twiddled stage-1 results through a private LDS
// buffer (no workgroup barrier).  The accumulators of its 512 pixels (8 per lane)
// stay in registers over the bins.  A workgroup is 8 waves = 16 depths of one frame;
// it stages each bin's coefficients and kz row in LDS (double-buffered, one barrier
// per bin).
//
// N = 512 splits the sum by the parity e of q first (radix 2 in frequency):
//     p(x) = P_0(x mod 256) + e^{2 pi i x / 512} P_1(x mod 256),
//     P_e(x') = sum_q' A(2 q' + e) e^{2 pi i q' x' / 256},
// and since e^{2 pi i (x' + 256) / 512} = -e^{2 pi i x' / 512}, the two pixels x' and
// x' + 256 are P_0 +- w P_1 with w = e^{2 pi i x' / 512}.  The two 256-point transforms
// of one depth take the place of the two depths in the tiles above (columns (q2, e)
// and (x1, e)), so a wave owns one depth and all 512 columns, and the lanes c and
// c ^ 16 that hold P_0(x') and P_1(x') exchange them for the combination.  With
// q' = 16 q1 + q2, coefficient q = 32 q1 + 2 q2 + e sits in staged row 2 q2 + e.
//
// Matrix-core operand layouts (lane l, h = l / 32, c = l % 32):
//   v_mfma_f32_32x32x2_f32:        A[c][2t + h],  B[2t + h][c],  t = 0..15 (k-steps)
//   v_mfma_f32_32x32x16_{bf16,f16}: A[c][16s + 8h + j], B[16s + 8h + j][c], s = 0..1, j = 0..7
//   result, register v = 0..15:     C[8(v/4) + 4h + v%4][c]
// K index <-> (input index m, re/im): FP32 k = 2t + h <-> m = 8h + t/2, re/im = t%2;
// 16-bit k = 16s + 8h + j <-> m = 8h + 4s + j/2, re/im = j%2.  Either way lane half h
// supplies the inputs m = 8h..8h+7 of its column, re and im.  Output rows are
// (x, re/im) = x + 16 (re/im), so register v < 8 holds Re and v + 8 Im of output
// x = 8(v/4) + 4h + v%4.
#pragma once
#include <type_traits>

#include "k3_fields16.hpp"

namespace pam {

constexpr int kFfN1 = 16;                 // stage-1 radix (and stage-3 radix at N = 256)
constexpr int kFfRow = 18;                // float2 pitch of a staged / transposed row of 16
constexpr int kFfZz = 16 * kFfRow + 16;   // float2 pitch of one depth's 16 rows in the transpose buffer
constexpr int kFfWaves = 8;               // waves per workgroup (2 / R depths each)

// depths per workgroup
template <int R>
__host__ __device__ constexpr int ff_depths() { return 2 * kFfWaves / R; }
// Staged inputs of one bin: G [NSUB][16 R rows][kFfRow] float2 then kz [16 R rows][kFfRow]
// doubles; row = q2 (R = 1) or 2 q2 + e (R = 2), 16 q1 per row.
template <int NSUB, int R>
__host__ __device__ constexpr int ff_stage_f2() { return (NSUB + 1) * 16 * R * kFfRow; }
// the same for N = 16 ROWS
template <int NSUB, int ROWS>
__host__ __device__ constexpr int ff_stage_rows() { return (NSUB + 1) * ROWS * kFfRow; }
// Transpose buffer of one wave: [NSUB][2 depths or halves][kFfZz] float2.
template <int NSUB>
__host__ __device__ constexpr int ff_tr_f2() { return NSUB * 2 * kFfZz; }
template <int NSUB, int R = 1>
inline size_t k3ff_lds() {
  return (size_t)(2 * ff_stage_f2<NSUB, R>() + kFfWaves * ff_tr_f2<NSUB>()) * sizeof(float2);
}

// Logical workgroup index (wg_group: XCD remap, group-local) -> (frame, depth tile, bin
// split).  Consecutive workgroups are dispatched round-robin over the 8 XCDs; the remap
// gives each XCD a contiguous range of logical indices, so the workgroups of one frame
// (which read the same per-bin coefficients) share one L2.
struct WgFF {
  int sp, dt, f, b_begin, b_end;
  __device__ WgFF(const K3Args& a, int bid) {
    sp = bid % a.n_split; bid /= a.n_split;
    dt = bid % a.n_dt;    bid /= a.n_dt;
    f = bid;
    b_begin = sp * a.bins_per_split;
    b_end = min(a.n_sel, b_begin + a.bins_per_split);
  }
};

// Element order of a bin's staged inputs for N = 16 ROWS: K2 writes a bin's coefficients of
// sub-aperture i in [i][row][q1] order and the kz table is [row][q1] (q = ROWS q1 + row), so
// 16-byte piece pi (two complex values or two doubles) is element 2 pi of that sequence; it
// lands in the stage buffer at rows of kFfRow float2.
template <int NSUB, int ROWS>
struct FfRows {
  static constexpr int NQ = 16 * ROWS;             // coefficients per sub-aperture
  static constexpr int NG = NSUB * NQ / 2;         // pieces of G
  static constexpr int PIECES = NG + NQ / 2;       // with the kz row
  static __device__ int where(int pi) {
    if (pi < NG) {
      const int e = 2 * pi, i = e / NQ, row = (e % NQ) >> 4, q1 = e & 15;
      return (i * ROWS + row) * kFfRow + q1;
    }
    if (pi < PIECES) {
      const int e = 2 * (pi - NG), row = e >> 4, q1 = e & 15;
      return NSUB * ROWS * kFfRow + row * kFfRow + q1;         // doubles at float2 granularity
    }
    return -1;
  }
  static __device__ uint4 fetch(const K3Args& a, int f, int b, int pi) {
    if (pi < NG) return *reinterpret_cast<const uint4*>(a.coeffs + ((size_t)f * a.n_sel + b) * NSUB * NQ + 2 * pi);
    return *reinterpret_cast<const uint4*>(a.kz_ff + (size_t)b * NQ + 2 * (pi - NG));
  }
};

// One 16-byte piece of a bin's staged inputs per thread and pass, R passes (512 R
// pieces cover NSUB <= 3): piece k of thread tid is piece tid + 512 k of FfRows.  The
// pieces are separate members (not an array) so that they stay in registers.
template <int NSUB, int R>
struct FfPiece {
  typedef FfRows<NSUB, 16 * R> P;
  uint4 v0, v1;
  int dst0, dst1;   // float2 offsets in the stage buffer, -1 for no piece
  static __device__ int where(int pi) { return P::where(pi); }
  static __device__ uint4 fetch(const K3Args& a, int f, int b, int pi) { return P::fetch(a, f, b, pi); }
  __device__ FfPiece(int tid) {
    dst0 = where(tid);
    dst1 = R > 1 ? where(tid + 512) : -1;
  }
  __device__ __forceinline__ void load(const K3Args& a, int f, int b, int tid) {
    if (dst0 >= 0) v0 = fetch(a, f, b, tid);
    if (R > 1 && dst1 >= 0) v1 = fetch(a, f, b, tid + 512);
  }
  __device__ __forceinline__ void store(float2* stage) const {
    if (dst0 >= 0) *reinterpret_cast<uint4*>(stage + dst0) = v0;
    if (R > 1 && dst1 >= 0) *reinterpret_cast<uint4*>(stage + dst1) = v1;
  }
};

// Twiddles e^{2 pi i q2 x1 / 256} of this lane's 8 stage-1 outputs (/ 16 for FP16 operands).
struct FfTw {
  float2 t[8];
  __device__ FfTw(const K3Args& a, int lane) {
    const float4* src = reinterpret_cast<const float4*>(a.ff_tw) + lane * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 q = src[k];
      t[2 * k] = make_float2(q.x, q.y);
      t[2 * k + 1] = make_float2(q.z, q.w);
    }
  }
};

// Combination twiddles e^{2 pi i x' / 512} of this lane's 8 stage-3 outputs (N = 512).
struct FfTw2 {
  float2 t[8];
  __device__ FfTw2() {}
  __device__ FfTw2(const K3Args& a, int lane) {
    const float4* src = reinterpret_cast<const float4*>(a.ff_tw2) + lane * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 q = src[k];
      t[2 * k] = make_float2(q.x, q.y);
      t[2 * k + 1] = make_float2(q.z, q.w);
    }
  }
};

// Lane (c, h) of a wave holds columns x = c%16 + 16 x2 (+ 256 for c >= 16 at N = 512),
// x2 = 8(v/4) + 4h + v%4 for v = 0..7, of depth d0 + c/16 (N = 256) or d0 (N = 512).
template <int NSUB, bool COH = false, int R = 1>
__device__ __forceinline__ void ff_store(const K3Args& a, int sp, int f, int d0, int lane,
                                         const float (&accS)[NSUB][8],
                                         const float (&accC)[AccCount<NSUB>::pairs > 0 ? AccCount<NSUB>::pairs : 1][8],
                                         const float (*accG)[8] = nullptr) {
  constexpr int NA = COH ? 5 : AccCount<NSUB>::total;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int N = 256 * R;
  const int c = lane & 31, h = lane >> 5;
  const int row = R == 1 ? d0 + (c >> 4) : d0;
  if (row >= a.n_z) return;
  const size_t plane = (size_t)a.n_z * N;
  float* dst = a.accum + ((size_t)sp * a.F + f) * NA * plane + (size_t)row * N + (c & 15) + (R == 1 ? 0 : 256 * (c >> 4));
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int x = 16 * (8 * (v >> 2) + 4 * h + (v & 3));
#pragma unroll
    for (int i = 0; i < NSUB; ++i) dst[i * plane + x] = accS[i][v];
#pragma unroll
    for (int p = 0; p < NP; ++p) dst[(NSUB + p) * plane + x] = accC[p][v];
    if constexpr (COH) {
#pragma unroll
      for (int g = 0; g < 4; ++g) dst[(1 + g) * plane + x] = accG[g][v];
    }
  }
}

// ---------------------------------------------------------------------------
// The kernel.  T = float: FP32 operands on v_mfma_f32_32x32x2_f32.  T = __bf16 or
// _Float16: operands on v_mfma_f32_32x32x16_*, each split into hi = T(x) and
// lo = T(x - hi); PASSES = 3 sums hi.hi + hi.lo + lo.hi, PASSES = 1 takes hi.hi.
//
// Per bin a wave runs a front half (propagator, stage-1 operands, stage-1
// products, twiddle, transpose into its LDS buffer) and a back half (stage-3
// operands from the buffer, stage-3 products, fold into the per-pixel sums).  The
// two waves that share a SIMD (w and w + 4) are half a bin apart: waves 0-3 run
// front(b) then back(b), waves 4-7 run back(b - 1) then front(b), so while one
// wave's products occupy the matrix core the other runs its VALU and LDS work.
//
// Scale: for FP16 operands K2 scales each bin's coefficients by a power of two s and
// the twiddles carry 1/16, so that both stages' operands stay in FP16 range; 16/s
// then multiplies the fields in the fold.  FP32 and BF16 operands take s = 1 and
// unscaled twiddles.
// ---------------------------------------------------------------------------
typedef float v2f __attribute__((ext_vector_type(2)));

template <typename T>
struct FfOps {
  typedef typename Mma<T>::v8 v8;
  typedef T v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float widen(T h) { return (float)h; }
  // 8 floats -> hi and lo 16-bit vectors, two values per conversion
  static __device__ __forceinline__ void split(const float (&x)[8], v8& hi, v8& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const v2f xx = {x[2 * j], x[2 * j + 1]};
      const v2 hh = __builtin_convertvector(xx, v2);
      const v2f back = __builtin_convertvector(hh, v2f);
      const v2 ll = __builtin_convertvector(xx - back, v2);
      hi[2 * j] = hh[0];
      hi[2 * j + 1] = hh[1];
      lo[2 * j] = ll[0];
      lo[2 * j + 1] = ll[1];
    }
  }
};

// COH (n_sub = 1 only): the back half also accumulates, per pixel, the cross-spectra
// with its lateral pair partner (column x ^ 1, the adjacent lane) and its axial pair
// partner (depth 2i <-> 2i + 1, the lane 16 away), G = sum over bins of p conj(p').
template <typename T, int PASSES, int NSUB, bool COH = false, int R = 1>
__global__ __launch_bounds__(512, 1) void k3ff(K3Args a0, K3Groups grp) {
  static_assert(!COH || (NSUB == 1 && R == 1), "pair cross-spectra come with the full-aperture sums at N = 256");
  static_assert(R == 1 || R == 2, "N = 256 or 512");
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr bool SCALED = std::is_same<T, _Float16>::value;   // keep K2's scale through stage 3
  constexpr int NP = AccCount<NSUB>::pairs;
  typedef typename std::conditional<F32, float, typename Mma<typename std::conditional<F32, __bf16, T>::type>::v8>::type v8;
  extern __shared__ float2 lds2[];
  float2* stage = lds2;                                          // [2][ff_stage_f2<NSUB, R>]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float2* tr = lds2 + 2 * ff_stage_f2<NSUB, R>() + w * ff_tr_f2<NSUB>();
  K3Args a = a0;
  const WgFF wg(a, wg_group(a, grp));
  const int f = wg.f;
  const int c = lane & 31, h = lane >> 5;
  // stage-1 column (q2, zz), stage-3 column (x1, zz): zz is the depth (N = 256) or the
  // parity e of q (N = 512)
  const int q2 = c & 15, zz = c >> 4;
  const int d0 = R == 1 ? wg.dt * ff_depths<R>() + 2 * w : wg.dt * ff_depths<R>() + w;
  const int depth = R == 1 ? d0 + zz : d0;
  const int srow = R == 1 ? q2 : 2 * q2 + zz;                    // staged row of this lane's inputs
  // rows beyond the grid run with z = 0: their pixels stay in their own columns of
  // both stages and are never stored
  const double z = depth < a.n_z ? a.z[depth] : 0.0;
  const bool lag = w >= 4;

  // constant 16-point DFT operands
  float W32[16];
  v8 Wh[2], Wl[2];
  if constexpr (F32) {
    const float4* src = reinterpret_cast<const float4*>(a.ff_w32) + lane * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 q = src[k];
      W32[4 * k] = q.x;
      W32[4 * k + 1] = q.y;
      W32[4 * k + 2] = q.z;
      W32[4 * k + 3] = q.w;
    }
  } else {
    const uint4* src = reinterpret_cast<const uint4*>(a.ff_w16) + lane * 4;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Wh[s] = __builtin_bit_cast(v8, src[2 * s]);
      Wl[s] = __builtin_bit_cast(v8, src[2 * s + 1]);
    }
  }
  const FfTw tw(a, lane);
  FfTw2 tw2;
  if constexpr (R == 2) tw2 = FfTw2(a, lane);
  float accS[NSUB][8];
  float accC[NP > 0 ? NP : 1][8];
  float accG[COH ? 4 : 1][8];      // Re, Im of the lateral, then of the axial pair sums
#pragma unroll
  for (int v = 0; v < 8; ++v) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[p][v] = 0.f;
#pragma unroll
    for (int g = 0; g < (COH ? 4 : 1); ++g) accG[g][v] = 0.f;
  }

  // products of one stage: C_i = W x operand_i for every sub-aperture
  auto gemm = [&](const float (&bf)[NSUB][16], const v8 (&bh)[NSUB][2], const v8 (&bl)[NSUB][2],
                  v16f (&C)[NSUB]) {
    // the first product of each chain takes a zero accumulator (an inline constant)
    const v16f zero = {};
    if constexpr (F32) {
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int i = 0; i < NSUB; ++i)
          C[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(W32[t], bf[i][t], t == 0 ? zero : C[i], 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < NSUB; ++i) {
          C[i] = Mma<T>::run(Wh[s], bh[i][s], s == 0 ? zero : C[i]);
          if (PASSES == 3) {
            C[i] = Mma<T>::run(Wh[s], bl[i][s], C[i]);
            C[i] = Mma<T>::run(Wl[s], bh[i][s], C[i]);
          }
        }
    }
  };
  // 16 operand values (inputs m = 8h..8h+7, re/im) of sub-aperture i into the operand registers
  auto put = [&](int i, const float (&x)[16], float (&bf)[NSUB][16], v8 (&bh)[NSUB][2], v8 (&bl)[NSUB][2]) {
    if constexpr (F32) {
#pragma unroll
      for (int t = 0; t < 16; ++t) bf[i][t] = x[t];
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        float y[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) y[j] = x[8 * s + j];
        FfOps<T>::split(y, bh[i][s], bl[i][s]);
      }
    }
  };

  // front half of bin b: stage-1 operands from the staged inputs, products, twiddle, transpose
  auto front = [&](int b) {
    const float2* st = stage + ((b - wg.b_begin) & 1) * ff_stage_f2<NSUB, R>();
    const double* kzr = reinterpret_cast<const double*>(st + NSUB * 16 * R * kFfRow) + srow * kFfRow + 8 * h;
    // propagator at the lane's 8 wavenumbers (Eq. 2): phase in FP64 reduced to
    // [-1/2, 1/2] cycle, hardware sin/cos; evanescent values (kz < 0 in the table) are
    // replaced in one branch taken only by lanes that hold any
    float2 H[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double ph = z * kzr[m];
      const float r = (float)(ph - rint(ph));
      H[m] = make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
    if (a.ev_bin[b]) {
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (kzr[m] < 0.0) H[m] = propagator(z, kzr[m], a.zero_evanescent);
    }
    float bf[NSUB][16];
    v8 bh[NSUB][2], bl[NSUB][2];
#pragma unroll
    for (int i = 0; i < NSUB; ++i) {
      const float4* g = reinterpret_cast<const float4*>(st + (i * 16 * R + srow) * kFfRow + 8 * h);
      float x[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 gg = g[k];
        const float2 a0 = cmul(H[2 * k], make_float2(gg.x, gg.y));
        const float2 a1 = cmul(H[2 * k + 1], make_float2(gg.z, gg.w));
        x[4 * k] = a0.x;
        x[4 * k + 1] = a0.y;
        x[4 * k + 2] = a1.x;
        x[4 * k + 3] = a1.y;
      }
      put(i, x, bf, bh, bl);
    }
    v16f C[NSUB];
    gemm(bf, bh, bl, C);
#pragma unroll
    for (int i = 0; i < NSUB; ++i)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int x1 = 8 * (v >> 2) + 4 * h + (v & 3);
        tr[i * 2 * kFfZz + zz * kFfZz + x1 * kFfRow + q2] = cmul(make_float2(C[i][v], C[i][v + 8]), tw.t[v]);
      }
    __builtin_amdgcn_wave_barrier();
  };

  // back half of bin b: stage-3 operands from the transpose buffer, products, fold
  auto back = [&](int b) {
    float bf[NSUB][16];
    v8 bh[NSUB][2], bl[NSUB][2];
#pragma unroll
    for (int i = 0; i < NSUB; ++i) {
      const float4* y = reinterpret_cast<const float4*>(tr + i * 2 * kFfZz + zz * kFfZz + q2 * kFfRow + 8 * h);
      float x[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 yy = y[k];
        x[4 * k] = yy.x;
        x[4 * k + 1] = yy.y;
        x[4 * k + 2] = yy.z;
        x[4 * k + 3] = yy.w;
      }
      put(i, x, bf, bh, bl);
    }
    v16f C[NSUB];
    gemm(bf, bh, bl, C);
    const float inv = SCALED ? 16.0f * a.inv_scale[(size_t)f * a.n_sel + b] : 1.0f;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      float pr[NSUB], pim[NSUB];
#pragma unroll
      for (int i = 0; i < NSUB; ++i) {
        pr[i] = SCALED ? C[i][v] * inv : C[i][v];
        pim[i] = SCALED ? C[i][v + 8] * inv : C[i][v + 8];
        if constexpr (R == 2) {
          // P_0 +- w P_1: lane half zz = 0 holds P_0(x'), zz = 1 P_1(x'), x' its column
          const float or_ = lane_xor16(pr[i]), oi = lane_xor16(pim[i]);
          const float2 p0 = zz ? make_float2(or_, oi) : make_float2(pr[i], pim[i]);
          const float2 p1 = zz ? make_float2(pr[i], pim[i]) : make_float2(or_, oi);
          const float2 t = cmul(tw2.t[v], p1);
          pr[i] = zz ? p0.x - t.x : p0.x + t.x;
          pim[i] = zz ? p0.y - t.y : p0.y + t.y;
        }
        accS[i][v] = fmaf(pr[i], pr[i], fmaf(pim[i], pim[i], accS[i][v]));
      }
      if constexpr (NSUB == 3) {
        accC[0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[0][v]));
        accC[1][v] = fmaf(pr[1], pr[2], fmaf(pim[1], pim[2], accC[1][v]));
        accC[2][v] = fmaf(pr[2], pr[0], fmaf(pim[2], pim[0], accC[2][v]));
      } else if constexpr (NSUB == 2) {
        accC[0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[0][v]));
      }
      if constexpr (COH) {
        // partner fields: column x ^ 1 sits in lane ^ 1, depth zz ^ 1 in lane ^ 16
        const float lr = lane_xor1(pr[0]), li = lane_xor1(pim[0]);
        const float zr = lane_xor16(pr[0]), zi = lane_xor16(pim[0]);
        accG[0][v] = fmaf(pr[0], lr, fmaf(pim[0], li, accG[0][v]));
        accG[1][v] = fmaf(pim[0], lr, fmaf(-pr[0], li, accG[1][v]));
        accG[2][v] = fmaf(pr[0], zr, fmaf(pim[0], zi, accG[2][v]));
        accG[3][v] = fmaf(pim[0], zr, fmaf(-pr[0], zi, accG[3][v]));
      }
    }
  };

  FfPiece<NSUB, R> pc(tid);
  if (wg.b_begin < wg.b_end) {
    pc.load(a, f, wg.b_begin, tid);
    pc.store(stage);
  }
  __syncthreads();
  // one extra iteration lets the lagging waves finish their last bin
  for (int b = wg.b_begin; b <= wg.b_end; ++b) {
    const bool has = b < wg.b_end, more = b + 1 < wg.b_end;
    if (more) pc.load(a, f, b + 1, tid);
    if (lag && b > wg.b_begin) back(b - 1);
    if (has) front(b);
    if (!lag && has) back(b);
    if (more) pc.store(stage + ((b + 1 - wg.b_begin) & 1) * ff_stage_f2<NSUB, R>());
    __syncthreads();
  }
  ff_store<NSUB, COH, R>(a, wg.sp, f, d0, lane, accS, accC, accG);
}

}  // namespace pam
