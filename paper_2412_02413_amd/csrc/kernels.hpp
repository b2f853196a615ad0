// Device kernels of the AS-TAX hot path for gfx950 (CDNA4, wave64).
//
//   k1_time_fft   F_t of every channel (Eq. 1): real FFT of n_t samples as an
//                 n_t/2-point complex Stockham FFT (radix 8) in LDS, then the in-band bins.
//   k2_lateral    apodization (Pattern-m masks) + lateral DFT F_x (Eq. 1) per
//                 (frame, bin), folded into the coefficients of a real DFT basis.
//   k3_fields     the propagator exp(i z kz) of Eq. 2 (FP64 phase, FP32 sin/cos)
//                 times the folded coefficients, the inverse lateral transform as
//                 a GEMM against a fixed real cos/sin basis on the matrix cores,
//                 and the sums over frequency of |p_i|^2 and Re(p_i^* p_j)
//                 (Eq. 4, Eq. 11) kept in registers.  Fields are never stored.
//   k4_weight     NCC pairs, eps floor, TAX cube root (Eq. 10), energy, per-block max.
//   k4_image      NNCC normalisation and I = rho_n^2 E (Eq. 11).
//
// Folding.  The propagator depends on kx only through kx^2, so H(q) = H(N-q) on
// the DFT grid.  Pairing q with N-q turns the inverse transform
//     p(x) = (1/N) sum_q H(q) P(q) e^{+2 pi i q x / N}
// into a sum over N real basis functions, cos(2 pi q x/N) for q = 0..N/2 and
// sin(2 pi q x/N) for q = 1..N/2-1, with complex coefficients
//     cos q:  H(q) (P(q) + P(N-q)) / N     (P(0)/N, P(N/2)/N at the ends)
//     sin q:  H(q) i (P(q) - P(N-q)) / N
// so each field is a complex-by-real product with K = N: half the work of the
// complex DFT and a basis matrix that is the same for every frame and bin.
// Slot order: slot 2q holds "cos q", slot 2q+1 holds "sin q" (slot 1 = cos N/2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pam {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Row pitch of the kz tables: N/2 + 1 values padded to an even count.
__host__ __device__ constexpr int kz_row(int N) { return N / 2 + 2; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// exp(i z kz) for one (depth, lateral wavenumber).  The table holds kz / (2 pi)
// in cycles per metre: kzc >= 0 is a propagating component, kzc < 0 encodes an
// evanescent one decaying as exp(2 pi z kzc).  The phase z*kz/(2 pi) (thousands
// of cycles at depth) is formed and reduced to [-1/2, 1/2] cycle in FP64; the
// sine and cosine of the reduced phase come from the hardware transcendental
// unit, whose argument is in cycles (max abs error ~1.2e-7 on [-1/2, 1/2]).  The
// decay exp(2 pi z kzc) = 2^(z kzc 2 pi / ln 2) comes from the hardware exp2.
constexpr float kTwoPiOverLn2 = 9.064720283654388f;
__device__ __forceinline__ float2 propagator(double z, double kzc, int zero_evanescent) {
  const double ph = z * kzc;
  if (kzc >= 0.0) {
    const float r = (float)(ph - rint(ph));
    return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
  }
  if (zero_evanescent) return make_float2(0.f, 0.f);
  return make_float2(__builtin_amdgcn_exp2f((float)ph * kTwoPiOverLn2), 0.f);
}

// --------------------------------------------------------------------------
// K1: time FFT.  One workgroup (256 threads) per (channel, frame).  The n_t real
// samples are read as M = n_t/2 complex values z[n] = x[2n] + i x[2n+1] and
// transformed by a Stockham auto-sort FFT: passes of radix 8 (then one of radix 4
// or 2 for the rest), each butterfly j of a pass reading z[j + r M/R], r < R,
// applying the twiddles e^{-2 pi i r k / (Ns R)} (k = j mod Ns, Ns = the size
// already transformed) and writing its R outputs at (j - k) R + k + r Ns, so the
// result lands in natural order with no bit reversal.  The first pass reads its
// operands straight from global memory (coalesced: consecutive threads take
// consecutive j); every pass keeps all of a thread's operands in registers
// between the workgroup barrier that ends the reads and the writes.  At 4096
// samples that is 4 passes instead of 11 radix-2 stages.  Finally
// X[k] = E[k] + e^{-2 pi i k/n_t} O[k] with E/O the transforms of the even/odd
// samples recovered from Z[k] and Z[M-k].
// --------------------------------------------------------------------------
struct K1Args {
  const float* rf;        // [F][L][n_t]
  float2* spectra;        // [F][n_sel][L]
  const float2* tw;       // e^{-2 pi i m / n_tp}, m < n_tp/2 (plan grid)
  const int32_t* ksel;    // bin k on the call's grid, [n_sel]
  int32_t L, n_t, log2m, tw_stride, n_sel;
  int32_t F;              // frames: the kernel walks the L F channels
};

// The value lane ^ 1 holds: DPP quad permutation [1, 0, 3, 2], a vector-ALU move.
__device__ __forceinline__ float lane_xor1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}
// The value lane ^ 16 holds: ds_swizzle in bit mode (and 0x1F, or 0, xor 0x10 within each
// 32 lanes), which moves data through the LDS crossbar without touching LDS memory.
__device__ __forceinline__ float lane_xor16(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}

// The value lane (16 - i) mod 16 of the lane's row of 16 holds (i = lane index in the row): a DPP row
// rotation by 15 (lane i takes lane i + 1 mod 16) followed by a DPP row mirror (lane i takes lane 15 - i).
__device__ __forceinline__ float lane_mirror16(float v) {
  const int t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x12F, 0xF, 0xF, false);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(t, 0x140, 0xF, 0xF, false));
}

// Rows 0 and 2 of the wave: the value lane (16 - i) mod 16 of the row holds, as lane_mirror16; rows 1 and 3: the
// value lane 15 - i holds.  The rotation is written to rows 0 and 2 only (DPP row mask 0b0101; the other rows keep
// their own values), then every row is mirrored.
__device__ __forceinline__ float lane_mirror16_odd_rows15(float v) {
  const int x = __builtin_bit_cast(int, v);
  const int t = __builtin_amdgcn_update_dpp(x, x, 0x12F, 0x5, 0xF, false);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(t, 0x140, 0xF, 0xF, false));
}

// Rows 2r and 2r + 1 of the wave as a pair: every lane i of both rows receives lane i of the even row in .x and
// lane i of the odd row in .y (v_permlane16_swap of a register with itself swaps the odd row of the first
// operand with the even row of the second).
__device__ __forceinline__ float2 rows_even_odd(float v) {
  const unsigned u = __builtin_bit_cast(unsigned, v);
  const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return make_float2(__builtin_bit_cast(float, (unsigned)r[0]), __builtin_bit_cast(float, (unsigned)r[1]));
}

// The value lane (8 - i) mod 8 of the lane's group of 8 holds (i = lane index in the group), for i = 1..7: the
// row rotation by 15 (lane i takes lane i + 1 mod 16) followed by a DPP half-row mirror (lane i takes lane 7 - i
// of its 8).  Lane 0 of each group receives a value from outside its group; callers use it only for i > 0.
__device__ __forceinline__ float lane_mirror8(float v) {
  const int t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x12F, 0xF, 0xF, false);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(t, 0x141, 0xF, 0xF, false));
}

__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // times -i

// in-place forward DFTs of 2, 4 and 8 points (e^{-2 pi i / R})
__device__ __forceinline__ void dft2(float2* v) {
  const float2 t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  const float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = mul_mi(csub(v1, v3));
  v0 = cadd(a0, a2);
  v2 = csub(a0, a2);
  v1 = cadd(a1, a3);
  v3 = csub(a1, a3);
}
__device__ __forceinline__ void dft8(float2* v) {
  // even and odd halves, then the radix-2 combination with w8^k, w8 = e^{-2 pi i / 8}
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const float r2 = 0.70710678118654752f;
  o1 = make_float2(r2 * (o1.x + o1.y), r2 * (o1.y - o1.x));        // (1 - i)/sqrt2
  o2 = mul_mi(o2);                                                    // -i
  o3 = make_float2(r2 * (o3.y - o3.x), -r2 * (o3.x + o3.y));       // (-1 - i)/sqrt2
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// LDS slot of point i of the K1 transform: one pad slot after every 8 points, so that the
// radix-8 pass writes (lane stride 8 points at NS = 1, runs of 8 at NS = 8) spread over
// the LDS banks instead of landing 8 to 16 lanes on one bank.
__device__ __forceinline__ int k1_slot(int i) { return i + (i >> 3); }
template <int M>
__host__ __device__ constexpr int k1_lds_points() { return M + M / 8; }

// One Stockham pass of radix R over M = 2^LOGM points, NS of them already transformed.
// EPT = elements per thread, so each thread runs EPT / R butterflies j = tid + 256 w.
// The first pass (NS = 1) takes its operands from registers v (loaded from global memory
// by k1_load), later passes from LDS.  Sizes and strides are compile-time constants, so
// the index arithmetic folds away and the pass needs few registers.
template <int LOGM, int R, int NS, int EPT>
__device__ __forceinline__ void k1_pass(float2 (&v)[EPT / R][R], float2* z, int tid) {
  constexpr int M = 1 << LOGM, NBF = M / R, PER = EPT / R;
  constexpr bool ALL = PER * 256 == NBF;   // every butterfly slot j = tid + 256 w is a butterfly
  if constexpr (NS > 1) {
#pragma unroll
    for (int w = 0; w < PER; ++w) {
      const int j = tid + 256 * w;
      if (ALL || j < NBF) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[w][r] = z[k1_slot(j + r * NBF)];
      }
    }
    __syncthreads();   // every read of this pass is done before any write
  }
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int j = tid + 256 * w;
    if (ALL || j < NBF) {
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
        // w1 = e^{-2 pi i k / (NS R)} from the hardware sine/cosine (argument in cycles,
        // an exact dyadic fraction), its higher powers by products
        const float c = (float)k * (1.0f / (float)(NS * R));
        const float2 w1 = make_float2(__builtin_amdgcn_cosf(c), -__builtin_amdgcn_sinf(c));
        float2 wr = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[w][r] = cmul(v[w][r], wr);
          if (r + 1 < R) wr = cmul(wr, w1);
        }
      }
      if constexpr (R == 8) dft8(v[w]);
      else if constexpr (R == 4) dft4(v[w][0], v[w][1], v[w][2], v[w][3]);
      else dft2(v[w]);
      const int idx = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) z[k1_slot(idx + r * NS)] = v[w][r];
    }
  }
  __syncthreads();
}

// Radix of the K1 pass at NS: 8 while at least 8 points remain, then 4 or 2.
template <int M, int NS>
__host__ __device__ constexpr int k1_radix() { return M / NS >= 8 ? 8 : (M / NS == 4 ? 4 : 2); }

// The passes after the first: NS = R0 onwards.
template <int LOGM, int NS, int EPT>
__device__ __forceinline__ void k1_passes(float2* z, int tid) {
  constexpr int M = 1 << LOGM;
  if constexpr (NS < M) {
    constexpr int R = k1_radix<M, NS>();
    float2 v[EPT / R][R];
    k1_pass<LOGM, R, NS, EPT>(v, z, tid);
    k1_passes<LOGM, NS * R, EPT>(z, tid);
  }
}

// The first pass's operands of one channel: butterfly j = tid + 256 w reads points
// j + r M / R0 (coalesced: consecutive threads take consecutive j).
template <int LOGM, int PER, int R>
__device__ __forceinline__ void k1_load(float2 (&v)[PER][R], const float2* src, int tid) {
  constexpr int M = 1 << LOGM, NBF = M / R;
  constexpr bool ALL = PER * 256 == NBF;
  static_assert(R == k1_radix<M, 1>(), "first-pass radix");
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int j = tid + 256 * w;
    if (ALL || j < NBF) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[w][r] = src[j + r * NBF];
    }
  }
}

// M = 2^LOGM = n_t / 2 complex points; EPT = elements per thread = max(8, M / 256).  A
// workgroup holds CH channels of one frame (elements l0 .. l0 + CH - 1), 256 threads and
// an LDS block per channel.  With CH = 2 a thread of the bin step writes one bin of both
// channels as one 16-byte store: half the store requests of one channel per workgroup,
// whose 8-byte stores each hit their own cache line (the bins of a channel lie L apart).
// Up to M = 2048 a thread holds 8 points and the kernel fits eight waves per SIMD.  Workgroup
// bid takes channel groups item = bid, bid + G, ... of the L F / CH (the host launches one
// group per workgroup, or fewer workgroups that each walk several); when it walks several,
// once the first pass has put a group into LDS the next group's samples are loaded into the
// registers it freed, so those HBM reads overlap the later LDS passes and the bin writes.  Consecutive workgroups go round-robin to the 8 XCDs, so the
// index is remapped to give each XCD runs of consecutive channel groups of a frame: their
// bin writes then fill the same cache lines of one L2.
template <int LOGM, int CH = 1, int EPT = (LOGM <= 11 ? 8 : (1 << LOGM) / 256)>
__global__ __launch_bounds__(256 * CH, EPT == 8 ? 8 : 2) void k1_time_fft(K1Args a) {
  extern __shared__ float2 k1_lds[];  // CH x [k1_lds_points<M>()], point i at k1_slot(i)
  constexpr int M = 1 << LOGM, R0 = k1_radix<M, 1>();
  static_assert(CH == 1 || (CH == 2 && EPT == 8), "two channels per workgroup up to 4096 samples");
  const int G = gridDim.x;
  int bid = blockIdx.x;
  if ((G & 7) == 0) bid = (bid & 7) * (G >> 3) + (bid >> 3);
  const int groups = a.L / CH;                 // channel groups per frame
  const int n_items = groups * a.F;
  const int sub = threadIdx.x >> 8, tid = threadIdx.x & 255;
  float2* z = k1_lds + sub * k1_lds_points<M>();
  float2 v[EPT / R0][R0];
  // channel of this thread's sub-group in group item: frame item / groups, element
  // (item % groups) CH + sub, i.e. row item CH + sub of [F][L]
  if (bid < n_items)
    k1_load<LOGM>(v, reinterpret_cast<const float2*>(a.rf + ((size_t)bid * CH + sub) * a.n_t), tid);
  for (int item = bid; item < n_items; item += G) {
    // the thread index, opaque to the compiler once per group: every twiddle and LDS
    // address derived from it is recomputed in each pass rather than hoisted out of the
    // loop and held in registers across it
    int t = tid;
    asm volatile("" : "+v"(t));
    k1_pass<LOGM, R0, 1, EPT>(v, z, t);       // consumes v
    if (item + G < n_items)                   // in flight during the remaining passes
      k1_load<LOGM>(v, reinterpret_cast<const float2*>(a.rf + ((size_t)(item + G) * CH + sub) * a.n_t), t);
    k1_passes<LOGM, R0, EPT>(z, t);
    const int l0 = (item % groups) * CH, f = item / groups;
    float2* dst = a.spectra + (size_t)f * a.n_sel * a.L + l0;
    // X[k] = E[k] + e^{-2 pi i k / n_t} O[k], E and O from Z[k] and conj Z[M - k]
    auto bin = [&](const float2* zz, int k, float2 w) {
      const float2 zk = zz[k1_slot(k)];
      const float2 zm = zz[k1_slot(M - k)];
      const float2 zc = make_float2(zm.x, -zm.y);
      const float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      const float2 d = csub(zk, zc);
      const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // (zk - zc) / (2i)
      return cadd(e, cmul(w, o));
    };
    if constexpr (CH == 1) {
      for (int b = t; b < a.n_sel; b += 256) {
        const int k = a.ksel[b];               // 0 < k < M
        dst[(size_t)b * a.L] = bin(z, k, a.tw[k * a.tw_stride]);
      }
    } else {
      // thread (b, pair): bin b of channels l0 + 2 pair and l0 + 2 pair + 1 (one pair)
      constexpr int PAIRS = CH / 2;
      for (int u = (int)threadIdx.x; u < PAIRS * a.n_sel; u += 256 * CH) {
        const int b = u / PAIRS, pr = u % PAIRS;
        const int k = a.ksel[b];
        const float2 w = a.tw[k * a.tw_stride];   // e^{-2 pi i k / n_t}
        const float2 x0 = bin(k1_lds + (2 * pr) * k1_lds_points<M>(), k, w);
        const float2 x1 = bin(k1_lds + (2 * pr + 1) * k1_lds_points<M>(), k, w);
        *reinterpret_cast<float4*>(dst + (size_t)b * a.L + 2 * pr) = make_float4(x0.x, x0.y, x1.x, x1.y);
      }
    }
    __syncthreads();                         // the next group's first pass overwrites z
  }
}

// --------------------------------------------------------------------------
// K2: apodize, place on the lateral grid, lateral DFT, fold into slot order (or,
// for the factored transform, reorder the unfolded spectrum so that q = N2 q1 + q2
// is stored at q2 N1 + q1) and scale by a power of two (exact) so that the largest
// coefficient lies in [2^11, 2^12) when the operands are FP16: this keeps FP16
// hi/lo splits of the products normal and is a no-op on the results (FP32 and BF16
// operands have the FP32 exponent range and take scale 1).  One workgroup per
// (bin, frame).
// --------------------------------------------------------------------------
struct K2Args {
  const float2* spectra;  // [F][n_sel][L]
  float2* coeffs;         // [F][n_sel][n_sub][N]
  float* inv_scale;       // [F][n_sel]
  const float2* twx;      // e^{-2 pi i m / N}, m < N
  const float* masks;     // [n_sub][L]
  int32_t L, N, n_sub, n_sel;
  int32_t col0, col_step; // grid column of element l is col0 + col_step * l
  int32_t ff_n1;          // 0: folded slot order; N1 > 0: unfolded P(q)/N in [q2][q1] order, q = (N/N1) q1 + q2
  int32_t scaled;         // 1: power-of-two scale into [2^11, 2^12) (FP16 operands); 0: scale 1
  int32_t n_items;        // F n_sel (one wave per (frame, bin) in k2_fft)
};

template <int NSUB>
__global__ __launch_bounds__(256) void k2_lateral(K2Args a) {
  extern __shared__ float2 sm2[];
  const int N = a.N;
  float2* tw = sm2;                   // [N]
  float2* u = tw + N;                 // [n_sub][L] apodized element spectra
  float2* P = u + 3 * a.L;            // [n_sub][N] lateral spectra
  float2* Gf = P + a.n_sub * N;       // [n_sub][N] folded coefficients
  __shared__ float red[256];
  const int b = blockIdx.x, f = blockIdx.y;
  const size_t fb = (size_t)f * a.n_sel + b;
  for (int m = threadIdx.x; m < N; m += blockDim.x) tw[m] = a.twx[m];
  for (int l = threadIdx.x; l < a.L; l += blockDim.x) {
    const float2 v = a.spectra[fb * a.L + l];
    for (int i = 0; i < a.n_sub; ++i) {
      const float mk = a.masks[i * a.L + l];
      u[i * a.L + l] = make_float2(mk * v.x, mk * v.y);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    float2 acc[NSUB];
#pragma unroll
    for (int i = 0; i < NSUB; ++i) acc[i] = make_float2(0.f, 0.f);
    // twiddle index (q * column) mod N, advanced by (q * col_step) mod N per element
    int m = (int)(((unsigned)q * (unsigned)a.col0) % (unsigned)N);
    const int dm = (int)(((unsigned)q * (unsigned)a.col_step) % (unsigned)N);
    for (int l = 0; l < a.L; ++l) {
      const float2 w = tw[m];
#pragma unroll
      for (int i = 0; i < NSUB; ++i) {
        const float2 v = u[i * a.L + l];
        acc[i].x = fmaf(v.x, w.x, fmaf(-v.y, w.y, acc[i].x));
        acc[i].y = fmaf(v.x, w.y, fmaf(v.y, w.x, acc[i].y));
      }
      m += dm;
      if (m >= N) m -= N;
    }
#pragma unroll
    for (int i = 0; i < NSUB; ++i) P[i * N + q] = acc[i];
  }
  __syncthreads();
  // fold into slot order and find the largest magnitude component
  const float invN = 1.0f / (float)N;
  float mx = 0.f;
  for (int e = threadIdx.x; e < a.n_sub * N; e += blockDim.x) {
    const int i = e / N, s = e - i * N, q = s >> 1;
    const float2* Pi = P + i * N;
    float2 g;
    if (a.ff_n1 > 0) {
      const int n2 = N / a.ff_n1;
      g = Pi[n2 * (s % a.ff_n1) + s / a.ff_n1];   // s = q2 N1 + q1
    } else if ((s & 1) == 0) {
      g = (q == 0) ? Pi[0] : cadd(Pi[q], Pi[N - q]);
    } else if (q == 0) {
      g = Pi[N / 2];
    } else {
      const float2 d = csub(Pi[q], Pi[N - q]);
      g = make_float2(-d.y, d.x);  // i (P(q) - P(N-q))
    }
    g.x *= invN;
    g.y *= invN;
    mx = fmaxf(mx, fmaxf(fabsf(g.x), fabsf(g.y)));
    Gf[e] = g;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  const float gmax = red[0];
  int ex = 0;
  frexpf(gmax, &ex);  // gmax = m 2^ex, m in [0.5, 1)
  const float scale = (a.scaled && gmax > 0.f) ? ldexpf(1.0f, 12 - ex) : 1.0f;
  float2* dst = a.coeffs + fb * a.n_sub * N;
  for (int e = threadIdx.x; e < a.n_sub * N; e += blockDim.x) {
    const float2 g = Gf[e];
    dst[e] = make_float2(g.x * scale, g.y * scale);
  }
  if (threadIdx.x == 0) a.inv_scale[fb] = 1.0f / scale;
}

// --------------------------------------------------------------------------
// K3 arguments (kernels in k3_fields.hpp).
// --------------------------------------------------------------------------
struct K3Args {
  const float2* coeffs;    // [F][n_sel][n_sub][N] slot order
  const float* inv_scale;  // [F][n_sel]
  const double* kz;        // [n_sel][kz_row(N)] signed kz / (2 pi) of the selected bins at q = 0..N/2, cycles per metre
  const double* z;         // [n_z]
  const float* basis;      // [N][N] slot-major fixed real basis (FP32 kernel)
  const void* basis_hi;    // [N/8 slot groups][N x][8 slots] basis, 16-bit hi part (split kernels)
  const void* basis_lo;    // same layout, 16-bit lo part
  float* accum;            // [n_split][F][n_acc][n_z][N]
  int32_t N, n_z, n_sel, F, n_dt, n_xg, n_split, bins_per_split, zero_evanescent;
  // factored-transform kernels (k3_factored.hpp)
  const double* kz_ff;     // [n_sel][N / 16][16] signed kz / (2 pi) at q = (N / 16) q1 + r, stored at [r][q1]
  const float* ff_w32;     // [64 lanes][16] 16-point DFT matrix, FP32 operand order
  const void* ff_w16;      // [64 lanes][2 k-steps][hi 8, lo 8] 16-point DFT matrix, 16-bit operand order
  const float2* ff_tw;     // [64 lanes][8] twiddles e^{2 pi i q2 x1 / N} of the lane's stage-1 outputs (/ 16 for FP16)
  const int32_t* ev_bin;   // [n_sel] 1 if the bin has evanescent lateral wavenumbers
  const float2* ff_tw2;    // [64 lanes][8] e^{2 pi i x' / 512} of the lane's stage-3 outputs (N = 512)
  const float2* ff_tw_vec; // [16 x1][16 q2] e^{2 pi i q2 x1 / 256} (vector FFT kernel)
  const float2* ff_tw2_vec; // [16 x2][16 j] e^{2 pi i (j + 16 x2) / 512} (vector FFT kernel, N = 512)
};

// Grouped work list of the factored fields kernels: frames of different record lengths
// (different bin sets) in one launch.  Group g owns workgroups [wg_begin, next wg_begin);
// its frames, bins and bin split replace the batch fields of K3Args.  n = 0: one batch.
constexpr int kMaxGroups = 8;
struct K3Group {
  const float2* coeffs;
  const float* inv_scale;
  const double* kz_ff;
  const int32_t* ev_bin;
  float* accum;
  int32_t wg_begin, F, n_sel, n_split, bins_per_split;
};
struct K3Groups {
  int32_t n;
  K3Group g[kMaxGroups];
};

// Workgroup index after the XCD remap (the workgroups of one logical range run on one XCD,
// so those of a frame share its L2); for a grouped launch the group's fields are patched
// into `a` and the index is made group-local.
__device__ __forceinline__ int wg_group(K3Args& a, const K3Groups& grp) {
  const int G = gridDim.x;
  int bid = blockIdx.x;
  // One frame batch: each XCD takes a contiguous eighth of the workgroups, so the tiles of a frame share one
  // L2.  A grouped launch keeps the hardware's round-robin order instead, so that every XCD gets the same mix
  // of the groups' (unequal) workgroups.
  if ((G & 7) == 0 && grp.n <= 1) bid = (bid & 7) * (G >> 3) + (bid >> 3);
  if (grp.n > 0) {
    int g = 0;
    while (g + 1 < grp.n && bid >= grp.g[g + 1].wg_begin) ++g;
    const K3Group& q = grp.g[g];
    a.coeffs = q.coeffs;
    a.inv_scale = q.inv_scale;
    a.kz_ff = q.kz_ff;
    a.ev_bin = q.ev_bin;
    a.accum = q.accum;
    a.F = q.F;
    a.n_sel = q.n_sel;
    a.n_split = q.n_split;
    a.bins_per_split = q.bins_per_split;
    bid -= q.wg_begin;
  }
  return bid;
}

template <int NSUB>
struct AccCount {
  static constexpr int pairs = NSUB == 3 ? 3 : (NSUB == 2 ? 1 : 0);
  static constexpr int total = NSUB + pairs;
};

// 16-bit matrix-core products used by the split-precision K3 kernels.
template <typename T>
struct Mma;
template <>
struct Mma<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ v16f run(v8 a, v8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ v16f run(v8 a, v8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <typename T>
struct Pair16 {
  T x, y;
};

// --------------------------------------------------------------------------
// K4: NCC, weight, energy, NNCC and image.
// --------------------------------------------------------------------------
struct K4Args {
  const float* accum;   // [n_split][F][n_acc][n_z][N]
  float* energy;        // [F][pix]
  float* weight;        // [F][pix]
  float* blockmax;      // [F][n_blk]
  float* rho_pairs;     // [F][n_pairs][pix] or null
  float* image;         // [F][pix]
  float* nncc;          // [F][pix] or null
  int32_t pix, F, n_split, n_sub, n_blk;
  int32_t n_acc;        // accumulator channels per frame (S, C and, with coherence, the pair sums)
  double eps;
};

__global__ __launch_bounds__(256) void k4_weight(K4Args a) {
  __shared__ float red[256];
  const int f = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int na = a.n_acc;                                        // channel stride
  const int nr = a.n_sub == 3 ? 6 : (a.n_sub == 2 ? 3 : 1);     // channels read here
  float wv = 0.f;
  if (p < a.pix) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < a.n_split; ++s) {
      const float* src = a.accum + ((size_t)s * a.F + f) * na * a.pix + p;
      for (int c = 0; c < nr; ++c) v[c] += (double)src[(size_t)c * a.pix];
    }
    double E, w;
    if (a.n_sub == 1) {
      E = v[0];
      w = 1.0;
    } else {
      const int np = a.n_sub == 3 ? 3 : 1;
      const int pi_[3] = {0, 1, 2}, pj_[3] = {1, 2, 0};
      double prod = 1.0, esum = 0.0;
      for (int i = 0; i < a.n_sub; ++i) esum += v[i];
      for (int q = 0; q < np; ++q) {
        const double cc = v[a.n_sub + q];
        esum += 2.0 * cc;
        const double den = sqrt(v[pi_[q]]) * sqrt(v[pj_[q]]);
        const double r = den > 0.0 ? cc / den : 0.0;
        if (a.rho_pairs) a.rho_pairs[((size_t)f * np + q) * a.pix + p] = (float)r;
        prod *= fmin(1.0, fmax(a.eps, r));
      }
      E = esum;
      w = (a.n_sub == 3) ? cbrt(prod) : prod;
    }
    a.energy[(size_t)f * a.pix + p] = (float)E;
    a.weight[(size_t)f * a.pix + p] = (float)w;
    wv = (float)w;
  }
  red[threadIdx.x] = wv;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.blockmax[(size_t)f * a.n_blk + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k4_image(K4Args a) {
  __shared__ float red[256];
  const int f = blockIdx.y;
  float m = 0.f;
  for (int i = threadIdx.x; i < a.n_blk; i += 256) m = fmaxf(m, a.blockmax[(size_t)f * a.n_blk + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  const float mx = red[0];
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < a.pix) {
    const size_t o = (size_t)f * a.pix + p;
    const float rn = a.weight[o] / mx;
    a.image[o] = rn * rn * a.energy[o];
    if (a.nncc) a.nncc[o] = rn;
  }
}

}  // namespace pam
