// K3 with 16-depth tiles on 16x16 matrix-core tiles.
//
// Same computation as k3_fields.hpp (propagator x folded coefficients, inverse
// lateral transform as a GEMM against the fixed real basis, per-bin folding of
// |p_i|^2 and Re(p_i^* p_j) into six per-pixel sums), with a different tiling:
// a workgroup owns one frame, 16 depths and 64*CT columns; each of its 4
// consumer waves owns CT 16x16 output tiles side by side (16 depths x 16 CT
// columns, 16 pixels per lane as in the 32x32 form).  Every generated A element
// therefore feeds 64*CT columns instead of 128, which halves the propagator
// work per matrix-core product at CT = 4, and each consumer wave reads 6 A
// rows-of-16 and CT B tiles per step instead of 6 A rows-of-32 and one B tile.
//
// Matrix-core layouts (16 x 16 output, lane l):
//   v_mfma_f32_16x16x4_f32:   A[l%16][l/16],        B[l/16][l%16]
//   v_mfma_f32_16x16x32_{bf16,f16}: A[l%16][8(l/16)+j], B[8(l/16)+j][l%16], j = 0..7
//   result v = 0..3:          C[4(l/16) + v][l%16]
#pragma once
#include "k3_fields.hpp"

namespace pam {

template <typename T>
struct Mma16;
template <>
struct Mma16<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ v4f run(v8 a, v8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma16<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ v4f run(v8 a, v8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Generation inputs of one stage for one producer thread (one slot pair of one row):
// kz / (2 pi) at the item's q and at q = N/2, the coefficients of slots 2q, 2q+1 of
// every sub-aperture, and the thread's share of the stage's basis tile.
template <int NSUB, typename BT, int CPY>
struct PairIn {
  double kz, kz_half;
  float4 g[NSUB];
  BT bc[CPY];
};

template <int NSUB, typename BT, int CPY>
__device__ __forceinline__ void load_pair_inputs(const K3Args& a, int f, int b, int q,
                                                 PairIn<NSUB, BT, CPY>& in) {
  const int N = a.N;
  const double* kzb = a.kz + (size_t)b * kz_row(N);
  in.kz = kzb[q];
  in.kz_half = kzb[N / 2];
  const float2* g = a.coeffs + ((size_t)f * a.n_sel + b) * NSUB * N;
#pragma unroll
  for (int i = 0; i < NSUB; ++i) in.g[i] = *reinterpret_cast<const float4*>(g + (size_t)i * N + 2 * q);
}

// vals[t][0..1] = A_t[r, 2ql], A_t[r, 2ql + 1] of tile t (Re / Im of each sub-aperture).
template <int NSUB, typename BT, int CPY>
__device__ __forceinline__ void gen_pair(const K3Args& a, double z, const PairIn<NSUB, BT, CPY>& in, bool q_is_zero,
                                         float vals[2 * NSUB][2]) {
  float2 h0 = make_float2(0.f, 0.f), h1 = h0;
  if (z >= 0.0) {
    h0 = propagator(z, in.kz, a.zero_evanescent);
    h1 = q_is_zero ? propagator(z, in.kz_half, a.zero_evanescent) : h0;
  }
#pragma unroll
  for (int i = 0; i < NSUB; ++i) {
    const float4 gg = in.g[i];
    const float2 a0 = cmul(h0, make_float2(gg.x, gg.y));
    const float2 a1 = cmul(h1, make_float2(gg.z, gg.w));
    vals[2 * i][0] = a0.x;
    vals[2 * i][1] = a1.x;
    vals[2 * i + 1][0] = a0.y;
    vals[2 * i + 1][1] = a1.y;
  }
}

template <int NSUB, int CT>
__device__ __forceinline__ void fold_bin16(const v4f (&C)[2 * NSUB][CT], float inv, float (&accS)[CT][NSUB][4],
                                           float (&accC)[CT][AccCount<NSUB>::pairs > 0 ? AccCount<NSUB>::pairs : 1][4]) {
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float pr[NSUB], pim[NSUB];
#pragma unroll
      for (int i = 0; i < NSUB; ++i) {
        pr[i] = C[2 * i][ct][v] * inv;
        pim[i] = C[2 * i + 1][ct][v] * inv;
        accS[ct][i][v] = fmaf(pr[i], pr[i], fmaf(pim[i], pim[i], accS[ct][i][v]));
      }
      if constexpr (NSUB == 3) {
        accC[ct][0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[ct][0][v]));
        accC[ct][1][v] = fmaf(pr[1], pr[2], fmaf(pim[1], pim[2], accC[ct][1][v]));
        accC[ct][2][v] = fmaf(pr[2], pr[0], fmaf(pim[2], pim[0], accC[ct][2][v]));
      } else if constexpr (NSUB == 2) {
        accC[ct][0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[ct][0][v]));
      }
    }
}

// Lane l of consumer wave w holds rows d0 + 4(l/16) + v and column x0 + 16 ct + l%16.
template <int NSUB, int CT>
__device__ __forceinline__ void store_acc16(const K3Args& a, int sp, int f, int d0, int x0, int lane,
                                            const float (&accS)[CT][NSUB][4],
                                            const float (&accC)[CT][AccCount<NSUB>::pairs > 0 ? AccCount<NSUB>::pairs : 1][4]) {
  constexpr int NA = AccCount<NSUB>::total;
  constexpr int NP = AccCount<NSUB>::pairs;
  const size_t plane = (size_t)a.n_z * a.N;
  float* dst = a.accum + ((size_t)sp * a.F + f) * NA * plane;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = d0 + 4 * (lane >> 4) + v;
      if (row < a.n_z) {
        const size_t o = (size_t)row * a.N + x0 + 16 * ct + (lane & 15);
#pragma unroll
        for (int i = 0; i < NSUB; ++i) dst[i * plane + o] = accS[ct][i][v];
#pragma unroll
        for (int p = 0; p < NP; ++p) dst[(NSUB + p) * plane + o] = accC[ct][p][v];
      }
    }
}

// Shared decode of the workgroup index and the stage range.
struct Wg16 {
  int sp, xg, dt, f, S;
  StageMap sm;
  __device__ Wg16(const K3Args& a, int kc) {
    int bid = blockIdx.x;
    sp = bid % a.n_split; bid /= a.n_split;
    xg = bid % a.n_xg;    bid /= a.n_xg;
    dt = bid % a.n_dt;    bid /= a.n_dt;
    f = bid;
    const int b_begin = sp * a.bins_per_split;
    const int b_end = min(a.n_sel, b_begin + a.bins_per_split);
    sm = StageMap{b_begin, a.N / kc};
    S = (b_end - b_begin) * sm.nch;
  }
};

// Producer pipeline shared by both kernels: inputs of stage s+2 are loaded while
// stage s+1 is generated, the two input sets alternate (no register copies), and
// loads are unconditional (the last stage's inputs are re-read past the end).
// One barrier per stage, matching the consumer loop: 1 + S barriers in total.
template <typename In, typename Load, typename Store>
__device__ __forceinline__ void produce(int S, In& cur, In& nxt, Load&& load, Store&& store) {
  if (S > 0) {
    load(0, cur);
    store(0, cur);
  }
  if (S > 1) load(1, cur);
  __syncthreads();
  auto step = [&](int s, In& gen, In& fill) {
    load(min(s + 2, S - 1), fill);
    store(s + 1, gen);
    __syncthreads();
  };
  int s = 0;
  for (; s + 2 < S; s += 2) {
    step(s, cur, nxt);
    step(s + 1, nxt, cur);
  }
  if (s + 1 < S) step(s, cur, nxt);
  if (S > 0) __syncthreads();   // stage S-1: nothing left to generate
}

// ---------------------------------------------------------------------------
// FP32 operands on v_mfma_f32_16x16x4_f32.
// LDS: A [2][2 NSUB][16 rows][34] floats (slot pairs adjacent; the 34-float row
// pitch keeps the producers' 8-byte stores and the consumers' 4-byte reads free
// of bank conflicts) and B [2][32 slots][64 CT + 16] floats.
// Producer thread p owns row p & 15 and slot pair p >> 4 of every stage.
// ---------------------------------------------------------------------------
template <int NSUB, int CT>
__global__ __launch_bounds__(512, 1) void k3f16_fp32(K3Args a) {
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int KC = 32, DR = 16, NC = 4, NPT = 256;
  constexpr int WCOLS = NC * CT * 16;
  constexpr int SP = KC + 2;
  constexpr int WCP = WCOLS + 16;
  constexpr int A_SZ = NT * DR * SP;
  constexpr int B_SZ = KC * WCP;
  constexpr int CPY = KC * WCOLS / 4 / NPT;
  static_assert(CPY >= 1 && (KC * WCOLS / 4) % NPT == 0, "basis copy split");
  extern __shared__ float smem[];
  float* Abuf = smem;
  float* Bbuf = smem + 2 * A_SZ;

  const Wg16 wg(a, KC);
  const int N = a.N, S = wg.S, f = wg.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d0 = wg.dt * DR, xwg = wg.xg * WCOLS;

  if (w >= NC) {
    const int ptid = tid - NC * 64;
    const int r = ptid & 15, ql = ptid >> 4;
    const double z = d0 + r < a.n_z ? a.z[d0 + r] : -1.0;
    typedef PairIn<NSUB, float4, CPY> In;
    In cur, nxt;
    auto load = [&](int s, In& in) {
      const int c = wg.sm.chunk(s);
      load_pair_inputs<NSUB>(a, f, wg.sm.bin(s), c * (KC / 2) + ql, in);
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        const int e = ptid + k * NPT;
        const int srow = e / (WCOLS / 4), c4 = e - srow * (WCOLS / 4);
        in.bc[k] = reinterpret_cast<const float4*>(a.basis + (size_t)(c * KC + srow) * N + xwg)[c4];
      }
    };
    auto store = [&](int s, const In& in) {
      float* Ab = Abuf + (s & 1) * A_SZ;
      float* Bb = Bbuf + (s & 1) * B_SZ;
      float vals[NT][2];
      gen_pair<NSUB>(a, z, in, wg.sm.chunk(s) == 0 && ql == 0, vals);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<float2*>(Ab + (t * DR + r) * SP + 2 * ql) = make_float2(vals[t][0], vals[t][1]);
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        const int e = ptid + k * NPT;
        const int srow = e / (WCOLS / 4), c4 = e - srow * (WCOLS / 4);
        *reinterpret_cast<float4*>(Bb + srow * WCP + 4 * c4) = in.bc[k];
      }
    };
    produce(S, cur, nxt, load, store);
    return;
  }

  // ---------------- consumer ----------------
  const int lr = lane & 15, lk = lane >> 4;
  const int xw = w * CT * 16;
  float accS[CT][NSUB][4];
  float accC[CT][NP > 0 ? NP : 1][4];
  v4f C[NT][CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int i = 0; i < NSUB; ++i) accS[ct][i][v] = 0.f;
#pragma unroll
      for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[ct][p][v] = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t) C[t][ct][v] = 0.f;
    }

  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const float* Ac = Abuf + (s & 1) * A_SZ;
    const float* Bc = Bbuf + (s & 1) * B_SZ;
    const bool last = wg.sm.chunk(s) == wg.sm.nch - 1;
    const float inv = last ? a.inv_scale[(size_t)f * a.n_sel + wg.sm.bin(s)] : 0.f;
#pragma unroll
    for (int j = 0; j < KC / 4; ++j) {
      float bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bv[ct] = Bc[(4 * j + lk) * WCP + xw + 16 * ct + lr];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float av = Ac[(t * DR + lr) * SP + 4 * j + lk];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) C[t][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], C[t][ct], 0, 0, 0);
      }
    }
    if (last) {
      fold_bin16<NSUB, CT>(C, inv, accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) C[t][ct][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc16<NSUB, CT>(a, wg.sp, f, d0, xwg + xw, lane, accS, accC);
}

// ---------------------------------------------------------------------------
// 16-bit operands on v_mfma_f32_16x16x32_{bf16,f16}: one matrix-core step per
// 32-slot stage.  Split x = hi + lo as in k3_fields_split (PASSES = 3: hi*hi +
// hi*lo + lo*hi; PASSES = 1: hi*hi).
// LDS: A [2][2 NSUB][hi, lo][16 rows][40] and B [2][hi, lo][64 CT][40] 16-bit.
// Producer thread p owns row p & 15 and slot pair p >> 4 of every stage.
// ---------------------------------------------------------------------------
template <typename T, int PASSES, int NSUB, int CT>
__global__ __launch_bounds__(512, 1) void k3f16_split(K3Args a) {
  typedef typename Mma16<T>::v8 v8;
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int KC = 32, DR = 16, NC = 4, NPT = 256;
  constexpr int RS = KC + 8;
  constexpr int WCOLS = NC * CT * 16;
  constexpr int NH = PASSES == 3 ? 2 : 1;
  constexpr int A_SZ = NT * NH * DR * RS;
  constexpr int B_SZ = NH * WCOLS * RS;
  constexpr int CPY = NH * WCOLS * (KC / 8) / NPT;
  static_assert(CPY >= 1 && (NH * WCOLS * (KC / 8)) % NPT == 0, "basis copy split");
  extern __shared__ float smem[];
  T* Abuf = reinterpret_cast<T*>(smem);
  T* Bbuf = Abuf + 2 * A_SZ;

  const Wg16 wg(a, KC);
  const int N = a.N, S = wg.S, f = wg.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d0 = wg.dt * DR, xwg = wg.xg * WCOLS;

  if (w >= NC) {
    const int ptid = tid - NC * 64;
    const int r = ptid & 15, ql = ptid >> 4;
    const double z = d0 + r < a.n_z ? a.z[d0 + r] : -1.0;
    typedef PairIn<NSUB, v8, CPY> In;
    In cur, nxt;
    // basis copy item e: column xc (fastest), 8-slot group g8, plane hl
    auto copy_item = [&](int k, int& xc, int& g8, int& hl) {
      const int e = ptid + k * NPT;
      xc = e % WCOLS;
      const int rest = e / WCOLS;
      g8 = rest % (KC / 8);
      hl = rest / (KC / 8);
    };
    auto load = [&](int s, In& in) {
      const int c = wg.sm.chunk(s);
      load_pair_inputs<NSUB>(a, f, wg.sm.bin(s), c * (KC / 2) + ql, in);
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        int xc, g8, hl;
        copy_item(k, xc, g8, hl);
        const T* src = reinterpret_cast<const T*>(hl ? a.basis_lo : a.basis_hi);
        in.bc[k] = *reinterpret_cast<const v8*>(src + ((size_t)(c * (KC / 8) + g8) * N + xwg + xc) * 8);
      }
    };
    auto store = [&](int s, const In& in) {
      T* Ab = Abuf + (s & 1) * A_SZ;
      T* Bb = Bbuf + (s & 1) * B_SZ;
      float vals[NT][2];
      gen_pair<NSUB>(a, z, in, wg.sm.chunk(s) == 0 && ql == 0, vals);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        Pair16<T> hi, lo;
        hi.x = (T)vals[t][0];
        hi.y = (T)vals[t][1];
        *reinterpret_cast<Pair16<T>*>(Ab + ((t * NH + 0) * DR + r) * RS + 2 * ql) = hi;
        if (NH == 2) {
          lo.x = (T)(vals[t][0] - (float)hi.x);
          lo.y = (T)(vals[t][1] - (float)hi.y);
          *reinterpret_cast<Pair16<T>*>(Ab + ((t * NH + 1) * DR + r) * RS + 2 * ql) = lo;
        }
      }
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        int xc, g8, hl;
        copy_item(k, xc, g8, hl);
        *reinterpret_cast<v8*>(Bb + (hl * WCOLS + xc) * RS + 8 * g8) = in.bc[k];
      }
    };
    produce(S, cur, nxt, load, store);
    return;
  }

  // ---------------- consumer ----------------
  const int lr = lane & 15, lk = lane >> 4;
  const int xw = w * CT * 16;
  float accS[CT][NSUB][4];
  float accC[CT][NP > 0 ? NP : 1][4];
  v4f C[NT][CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int i = 0; i < NSUB; ++i) accS[ct][i][v] = 0.f;
#pragma unroll
      for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[ct][p][v] = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t) C[t][ct][v] = 0.f;
    }

  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const T* Ac = Abuf + (s & 1) * A_SZ;
    const T* Bc = Bbuf + (s & 1) * B_SZ;
    const bool last = wg.sm.chunk(s) == wg.sm.nch - 1;
    const float inv = last ? a.inv_scale[(size_t)f * a.n_sel + wg.sm.bin(s)] : 0.f;
    v8 bh[CT], bl[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      bh[ct] = *reinterpret_cast<const v8*>(Bc + (0 * WCOLS + xw + 16 * ct + lr) * RS + 8 * lk);
      if (NH == 2) bl[ct] = *reinterpret_cast<const v8*>(Bc + (1 * WCOLS + xw + 16 * ct + lr) * RS + 8 * lk);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const v8 ah = *reinterpret_cast<const v8*>(Ac + ((t * NH + 0) * DR + lr) * RS + 8 * lk);
      v8 al;
      if (NH == 2) al = *reinterpret_cast<const v8*>(Ac + ((t * NH + 1) * DR + lr) * RS + 8 * lk);
      // pass-major order: consecutive products update different accumulators
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) C[t][ct] = Mma16<T>::run(ah, bh[ct], C[t][ct]);
      if (NH == 2) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) C[t][ct] = Mma16<T>::run(ah, bl[ct], C[t][ct]);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) C[t][ct] = Mma16<T>::run(al, bh[ct], C[t][ct]);
      }
    }
    if (last) {
      fold_bin16<NSUB, CT>(C, inv, accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) C[t][ct][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc16<NSUB, CT>(a, wg.sp, f, d0, xwg + xw, lane, accS, accC);
}

// LDS bytes of the kernels above
template <int NSUB, int CT>
constexpr size_t k3f16_fp32_lds() {
  return (size_t)2 * ((2 * NSUB) * 16 * 34 + 32 * (64 * CT + 16)) * sizeof(float);
}
template <int PASSES, int NSUB, int CT>
constexpr size_t k3f16_split_lds() {
  return (size_t)2 * ((2 * NSUB) * (PASSES == 3 ? 2 : 1) * 16 * 40 + (PASSES == 3 ? 2 : 1) * 64 * CT * 40) * 2;
}

}  // namespace pam
