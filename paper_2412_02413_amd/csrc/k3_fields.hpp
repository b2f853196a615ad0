// K3: fused propagate + inverse lateral transform (DFT-GEMM on the matrix cores)
// + sums over frequency of the sub-aperture cross-spectra.
//
// GEMM view for one (frame, bin): rows = depths, K = N slots, columns = x.
//   A_t[d, s] = Re or Im of H(d, q(s)) * coeff_i[s]      (t = 2 i + {0: re, 1: im})
//   B[s, x]   = fixed real basis (slot 2q: cos 2 pi q x / N, slot 2q+1: sin, slot 1: cos pi x)
//   p_i(d, x) = (A_{2i} B)(d, x) + i (A_{2i+1} B)(d, x)
// H(d, q) = exp(i z_d kz(q)) is Eq. 2's propagator; the fields p_i are the
// monochromatic fields of each sub-aperture at every pixel.  Per bin, each pixel's
// |p_i|^2 and Re(p_i^* p_j) (Eq. 4 with conjugate negative frequencies, Appendix A)
// are added to six FP32 accumulators held in registers; fields are never stored.
//
// Work decomposition.  A workgroup owns one frame, one 32-depth tile, NC*32
// columns (one 32-column tile per consumer wave) and a contiguous range
// of bins.  The (bin, K-chunk) pairs of that range form a pipeline of stages:
// while the consumer waves run the matrix cores on stage s out of LDS buffer s&1,
// the producer waves generate the A tile of stage s+1 (FP64 phase and reduction,
// FP32 sin/cos, complex product with the coefficients) and copy the basis tile
// of stage s+1 from L2 into buffer (s+1)&1.  One barrier per stage.  Each A element
// is made once per workgroup and reused by every consumer wave.
#pragma once
#include "kernels.hpp"

namespace pam {

// Stage geometry shared by the FP32 and 16-bit kernels.
struct StageMap {
  int b_begin, nch;
  __device__ __forceinline__ int bin(int s) const { return b_begin + s / nch; }
  __device__ __forceinline__ int chunk(int s) const { return s - (s / nch) * nch; }
};

// Generation items.  Producer thread ptid owns items e = ptid + k * npt of every
// stage: row r = e & 31 of the depth tile and slot pair ql = e >> 5 (slots 2ql and
// 2ql + 1 of the stage's chunk).  The row, hence the depth, is fixed across stages;
// a negative depth marks a row beyond the grid (zero propagator).
template <int GEN>
struct GenRows {
  double z[GEN];
  __device__ GenRows(const K3Args& a, int ptid, int npt, int d0) {
#pragma unroll
    for (int k = 0; k < GEN; ++k) {
      const int d = d0 + ((ptid + k * npt) & 31);
      z[k] = d < a.n_z ? a.z[d] : -1.0;
    }
  }
};

// Global inputs of one stage for one producer thread: kz / (2 pi) at each item's q,
// at q = N/2 (slot 1 holds cos(pi x)), the coefficients of slots 2q, 2q+1 of every
// sub-aperture, and the thread's share of the stage's basis tile.
template <int NSUB, int GEN, typename BT, int CPY>
struct StageIn {
  double kz[GEN];
  double kz_half;
  float4 g[GEN][NSUB];
  BT bc[CPY];
};

template <int NSUB, int GEN, typename BT, int CPY>
__device__ __forceinline__ void load_gen_inputs(const K3Args& a, int f, int b, int q0, int ptid, int npt,
                                                StageIn<NSUB, GEN, BT, CPY>& in) {
  const int N = a.N;
  const double* kzb = a.kz + (size_t)b * kz_row(N);
  in.kz_half = kzb[N / 2];
  const float2* g = a.coeffs + ((size_t)f * a.n_sel + b) * NSUB * N;
#pragma unroll
  for (int k = 0; k < GEN; ++k) {
    const int q = q0 + ((ptid + k * npt) >> 5);
    in.kz[k] = kzb[q];
#pragma unroll
    for (int i = 0; i < NSUB; ++i) in.g[k][i] = *reinterpret_cast<const float4*>(g + (size_t)i * N + 2 * q);
  }
}

// A values of item k: vals[t][0..1] = A_t[r, 2ql], A_t[r, 2ql + 1] for every tile t.
template <int NSUB, int GEN, typename BT, int CPY>
__device__ __forceinline__ void gen_values(const K3Args& a, double z, const StageIn<NSUB, GEN, BT, CPY>& in, int k,
                                           bool q_is_zero, float vals[2 * NSUB][2]) {
  float2 h0 = make_float2(0.f, 0.f), h1 = h0;
  if (z >= 0.0) {
    h0 = propagator(z, in.kz[k], a.zero_evanescent);
    h1 = q_is_zero ? propagator(z, in.kz_half, a.zero_evanescent) : h0;
  }
#pragma unroll
  for (int i = 0; i < NSUB; ++i) {
    const float4 gg = in.g[k][i];
    const float2 a0 = cmul(h0, make_float2(gg.x, gg.y));
    const float2 a1 = cmul(h1, make_float2(gg.z, gg.w));
    vals[2 * i][0] = a0.x;
    vals[2 * i][1] = a1.x;
    vals[2 * i + 1][0] = a0.y;
    vals[2 * i + 1][1] = a1.y;
  }
}

template <int NSUB, int XT>
__device__ __forceinline__ void fold_bin(const v16f (&C)[XT][2 * NSUB], float inv,
                                         float (&accS)[XT][NSUB][16],
                                         float (&accC)[XT][AccCount<NSUB>::pairs > 0 ? AccCount<NSUB>::pairs : 1][16]) {
#pragma unroll
  for (int xt = 0; xt < XT; ++xt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float pr[NSUB], pim[NSUB];
#pragma unroll
      for (int i = 0; i < NSUB; ++i) {
        pr[i] = C[xt][2 * i][v] * inv;
        pim[i] = C[xt][2 * i + 1][v] * inv;
        accS[xt][i][v] = fmaf(pr[i], pr[i], fmaf(pim[i], pim[i], accS[xt][i][v]));
      }
      if constexpr (NSUB == 3) {
        accC[xt][0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[xt][0][v]));
        accC[xt][1][v] = fmaf(pr[1], pr[2], fmaf(pim[1], pim[2], accC[xt][1][v]));
        accC[xt][2][v] = fmaf(pr[2], pr[0], fmaf(pim[2], pim[0], accC[xt][2][v]));
      } else if constexpr (NSUB == 2) {
        accC[xt][0][v] = fmaf(pr[0], pr[1], fmaf(pim[0], pim[1], accC[xt][0][v]));
      }
    }
}

// 32x32 accumulator layout: lane holds column (lane & 31) and rows
// 8*(v/4) + 4*(lane/32) + v%4 for v = 0..15.
template <int NSUB, int XT>
__device__ __forceinline__ void store_acc(const K3Args& a, int sp, int f, int d0, int xw, int lane,
                                          const float (&accS)[XT][NSUB][16],
                                          const float (&accC)[XT][AccCount<NSUB>::pairs > 0 ? AccCount<NSUB>::pairs : 1][16]) {
  constexpr int NA = AccCount<NSUB>::total;
  constexpr int NP = AccCount<NSUB>::pairs;
  const int N = a.N;
  const size_t plane = (size_t)a.n_z * N;
  float* dst = a.accum + ((size_t)sp * a.F + f) * NA * plane;
  const int half = lane >> 5, col = lane & 31;
#pragma unroll
  for (int xt = 0; xt < XT; ++xt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = d0 + 8 * (v >> 2) + 4 * half + (v & 3);
      if (row < a.n_z) {
        const size_t o = (size_t)row * N + xw + xt * 32 + col;
#pragma unroll
        for (int i = 0; i < NSUB; ++i) dst[i * plane + o] = accS[xt][i][v];
#pragma unroll
        for (int p = 0; p < NP; ++p) dst[(NSUB + p) * plane + o] = accC[xt][p][v];
      }
    }
}

// ---------------------------------------------------------------------------
// Wave roles.  A workgroup has 2*NC waves: waves 0..NC-1 are consumers (one
// 32x32 output tile each, matrix-core products only, operands from LDS),
// waves NC..2NC-1 are producers (propagator generation and basis copy for
// the next stage).  With one workgroup per CU each SIMD runs one consumer and
// one producer, so the generation's VALU work and memory latency overlap the
// matrix cores.  Both roles run the same number of barriers (one per stage);
// their loops are separate so the consumers' 192 accumulator registers are not
// live in the producer code.
// ---------------------------------------------------------------------------

// FP32 operands on v_mfma_f32_32x32x2_f32 (K = 2 slots per instruction).
// LDS: A [2][2 NSUB][KC][32] and B [2][KC][WC] floats.
template <int NSUB, int NC>
__global__ __launch_bounds__(NC * 128, 1) void k3_fields_fp32(K3Args a) {
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int KC = 32;
  constexpr int WC = NC * 32;
  constexpr int NPT = NC * 64;                 // producer threads
  constexpr int A_SZ = NT * KC * 32;
  constexpr int B_SZ = KC * WC;
  constexpr int GEN = 32 * (KC / 2) / NPT;     // generation items per producer thread per stage
  constexpr int CPY = (KC * WC / 4) / NPT;     // float4 basis copies per producer thread per stage
  static_assert(GEN >= 1 && (32 * (KC / 2)) % NPT == 0, "generation split");
  static_assert(CPY >= 1 && (KC * WC / 4) % NPT == 0, "basis copy split");
  extern __shared__ float smem[];
  float* Abuf = smem;                 // [2][A_SZ]
  float* Bbuf = smem + 2 * A_SZ;      // [2][B_SZ]

  const int N = a.N;
  int bid = blockIdx.x;
  const int sp = bid % a.n_split; bid /= a.n_split;
  const int xg = bid % a.n_xg;    bid /= a.n_xg;
  const int dt = bid % a.n_dt;    bid /= a.n_dt;
  const int f = bid;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int xwg = xg * WC;
  const int d0 = dt * 32;
  const int b_begin = sp * a.bins_per_split;
  const int b_end = min(a.n_sel, b_begin + a.bins_per_split);
  const StageMap sm{b_begin, N / KC};
  const int S = (b_end - b_begin) * sm.nch;

  if (w >= NC) {
    // ---------------- producer ----------------
    const int ptid = tid - NC * 64;
    const GenRows<GEN> rows(a, ptid, NPT, d0);
    StageIn<NSUB, GEN, float4, CPY> cur, nxt;
    auto load = [&](int s, StageIn<NSUB, GEN, float4, CPY>& in) {
      const int c = sm.chunk(s);
      load_gen_inputs<NSUB, GEN>(a, f, sm.bin(s), c * (KC / 2), ptid, NPT, in);
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        const int e = ptid + k * NPT;
        const int row = e / (WC / 4), c4 = e - row * (WC / 4);
        in.bc[k] = reinterpret_cast<const float4*>(a.basis + (size_t)(c * KC + row) * N + xwg)[c4];
      }
    };
    auto store = [&](int s, const StageIn<NSUB, GEN, float4, CPY>& in, float* Ab, float4* Bb) {
      const int c0q = sm.chunk(s) * (KC / 2);
#pragma unroll
      for (int k = 0; k < GEN; ++k) {
        const int e = ptid + k * NPT;
        const int r = e & 31, ql = e >> 5;
        float vals[NT][2];
        gen_values<NSUB>(a, rows.z[k], in, k, c0q + ql == 0, vals);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          Ab[(t * KC + 2 * ql) * 32 + r] = vals[t][0];
          Ab[(t * KC + 2 * ql + 1) * 32 + r] = vals[t][1];
        }
      }
#pragma unroll
      for (int k = 0; k < CPY; ++k) Bb[ptid + k * NPT] = in.bc[k];
    };
    // inputs of stage s+2 are in flight while stage s+1 is generated; the two
    // input sets swap roles every stage (no register copies, so no wait on loads
    // still in flight)
    if (S > 0) {
      load(0, cur);
      store(0, cur, Abuf, reinterpret_cast<float4*>(Bbuf));
    }
    if (S > 1) load(1, cur);
    __syncthreads();
    // Loads are unconditional (the last stage's inputs are re-read past the end) so
    // the in-flight registers never merge with older values at a branch.
    auto step = [&](int s, StageIn<NSUB, GEN, float4, CPY>& gen, StageIn<NSUB, GEN, float4, CPY>& fill) {
      load(min(s + 2, S - 1), fill);
      store(s + 1, gen, Abuf + ((s + 1) & 1) * A_SZ, reinterpret_cast<float4*>(Bbuf + ((s + 1) & 1) * B_SZ));
      __syncthreads();
    };
    int s = 0;
    for (; s + 2 < S; s += 2) {
      step(s, cur, nxt);
      step(s + 1, nxt, cur);
    }
    if (s + 1 < S) {
      step(s, cur, nxt);
      ++s;
    }
    if (S > 0) __syncthreads();   // stage S-1: nothing left to generate
    return;
  }

  // ---------------- consumer ----------------
  const int half = lane >> 5, col = lane & 31;
  float accS[1][NSUB][16];
  float accC[1][NP > 0 ? NP : 1][16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[0][i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[0][p][v] = 0.f;
  }
  v16f C[1][NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;

  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const float* Ac = Abuf + (s & 1) * A_SZ;
    const float* Bc = Bbuf + (s & 1) * B_SZ;
#pragma unroll
    for (int j = 0; j < KC / 2; ++j) {
      const float bv = Bc[(2 * j + half) * WC + w * 32 + col];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float av = Ac[(t * KC + 2 * j + half) * 32 + col];
        C[0][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, C[0][t], 0, 0, 0);
      }
    }
    if (sm.chunk(s) == sm.nch - 1) {
      fold_bin<NSUB, 1>(C, a.inv_scale[(size_t)f * a.n_sel + sm.bin(s)], accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc<NSUB, 1>(a, sp, f, d0, xwg + w * 32, lane, accS, accC);
}

// Generation items of the 16-bit kernels: four consecutive slots (two slot
// pairs) of one row, so each A plane is written with one 8-byte LDS store per
// item.  Item e: slot quad p4 = (e & 1) | ((e >> 6) << 1), row r = (e >> 1) & 31.
// Within 16 lanes this covers 8 rows x 2 quads, whose 8-byte stores fall in
// distinct banks for the 80-byte row pitch.
struct QuadItem {
  int r, p4;
  __device__ QuadItem(int e) : r((e >> 1) & 31), p4((e & 1) | ((e >> 6) << 1)) {}
};

template <int NSUB, int GENQ, typename BT, int CPY>
struct QuadIn {
  double2 kz[GENQ];        // kz / (2 pi) at q and q + 1
  double kz_half;
  float4 g[GENQ][NSUB][2];  // coefficients of the quad's four slots
  BT bc[CPY];
};

template <int NSUB, int GENQ, typename BT, int CPY>
__device__ __forceinline__ void load_quad_inputs(const K3Args& a, int f, int b, int q0, int ptid, int npt,
                                                 QuadIn<NSUB, GENQ, BT, CPY>& in) {
  const int N = a.N;
  const double* kzb = a.kz + (size_t)b * kz_row(N);   // even row pitch: 16-byte aligned pairs
  in.kz_half = kzb[N / 2];
  const float2* g = a.coeffs + ((size_t)f * a.n_sel + b) * NSUB * N;
#pragma unroll
  for (int k = 0; k < GENQ; ++k) {
    const QuadItem it(ptid + k * npt);
    const int q = q0 + 2 * it.p4;            // q0 even, so q is even: 16-byte aligned pair
    in.kz[k] = *reinterpret_cast<const double2*>(kzb + q);
#pragma unroll
    for (int i = 0; i < NSUB; ++i) {
      const float4* gp = reinterpret_cast<const float4*>(g + (size_t)i * N + 2 * q);
      in.g[k][i][0] = gp[0];
      in.g[k][i][1] = gp[1];
    }
  }
}

// A values of quad item k: vals[t][j] = A_t[r, 4 p4 + j] for every tile t.
template <int NSUB, int GENQ, typename BT, int CPY>
__device__ __forceinline__ void gen_quad(const K3Args& a, double z, const QuadIn<NSUB, GENQ, BT, CPY>& in, int k,
                                         bool q_is_zero, float vals[2 * NSUB][4]) {
  float2 h0 = make_float2(0.f, 0.f), h1 = h0, h2 = h0;
  if (z >= 0.0) {
    h0 = propagator(z, in.kz[k].x, a.zero_evanescent);
    h1 = q_is_zero ? propagator(z, in.kz_half, a.zero_evanescent) : h0;
    h2 = propagator(z, in.kz[k].y, a.zero_evanescent);
  }
#pragma unroll
  for (int i = 0; i < NSUB; ++i) {
    const float4 g0 = in.g[k][i][0], g1 = in.g[k][i][1];
    const float2 a0 = cmul(h0, make_float2(g0.x, g0.y));
    const float2 a1 = cmul(h1, make_float2(g0.z, g0.w));
    const float2 a2 = cmul(h2, make_float2(g1.x, g1.y));
    const float2 a3 = cmul(h2, make_float2(g1.z, g1.w));
    vals[2 * i][0] = a0.x;
    vals[2 * i][1] = a1.x;
    vals[2 * i][2] = a2.x;
    vals[2 * i][3] = a3.x;
    vals[2 * i + 1][0] = a0.y;
    vals[2 * i + 1][1] = a1.y;
    vals[2 * i + 1][2] = a2.y;
    vals[2 * i + 1][3] = a3.y;
  }
}

template <typename T>
struct alignas(8) Quad16 {
  T v[4];
};

// 16-bit operands on v_mfma_f32_32x32x16_{bf16,f16} (K = 16 slots per
// instruction).  Operands are split x = hi + lo (hi = round16(x),
// lo = round16(x - hi)); PASSES = 3 accumulates hi*hi + hi*lo + lo*hi in FP32
// (lo*lo lies below the FP32 rounding of the sum), PASSES = 1 keeps hi*hi.
// FP16 relies on the power-of-two pre-scaling of the coefficients (largest
// in [2^11, 2^12)), which keeps products in range and significant lo parts normal.
// LDS: A [2][2 NSUB][hi, lo][32][KC + 8] and B [2][hi, lo][WC][KC + 8] 16-bit
// (8-element row padding against bank conflicts on 16-byte reads).
template <typename T, int PASSES, int NSUB, int NC>
__global__ __launch_bounds__(NC * 128, 1) void k3_fields_split(K3Args a) {
  typedef typename Mma<T>::v8 v8;
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int KC = 32;
  constexpr int RS = KC + 8;
  constexpr int WC = NC * 32;
  constexpr int NPT = NC * 64;
  constexpr int NH = PASSES == 3 ? 2 : 1;   // hi (and lo) planes
  constexpr int A_SZ = NT * NH * 32 * RS;   // elements
  constexpr int B_SZ = NH * WC * RS;
  constexpr int GENQ = 32 * (KC / 4) / NPT;         // quad items per producer thread per stage
  constexpr int CPY = (NH * WC * (KC / 8)) / NPT;   // 16-byte basis copies per producer thread
  static_assert(GENQ >= 1 && (32 * (KC / 4)) % NPT == 0, "generation split");
  static_assert(CPY >= 1 && (NH * WC * (KC / 8)) % NPT == 0, "basis copy split");
  extern __shared__ float smem[];
  T* Abuf = reinterpret_cast<T*>(smem);     // [2][A_SZ]
  T* Bbuf = Abuf + 2 * A_SZ;                // [2][B_SZ]

  const int N = a.N;
  int bid = blockIdx.x;
  const int sp = bid % a.n_split; bid /= a.n_split;
  const int xg = bid % a.n_xg;    bid /= a.n_xg;
  const int dt = bid % a.n_dt;    bid /= a.n_dt;
  const int f = bid;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int xwg = xg * WC;
  const int d0 = dt * 32;
  const int b_begin = sp * a.bins_per_split;
  const int b_end = min(a.n_sel, b_begin + a.bins_per_split);
  const StageMap sm{b_begin, N / KC};
  const int S = (b_end - b_begin) * sm.nch;

  if (w >= NC) {
    // ---------------- producer ----------------
    const int ptid = tid - NC * 64;
    double zr[GENQ];
#pragma unroll
    for (int k = 0; k < GENQ; ++k) {
      const int d = d0 + QuadItem(ptid + k * NPT).r;
      zr[k] = d < a.n_z ? a.z[d] : -1.0;
    }
    QuadIn<NSUB, GENQ, v8, CPY> cur, nxt;
    // basis copy item e: column xc (fastest, so 8 lanes of one 16-byte store
    // group hit 8 distinct bank groups for the 80-byte pitch), 8-slot group g8, plane hl
    auto copy_item = [&](int k, int& xc, int& g8, int& hl) {
      const int e = ptid + k * NPT;
      xc = e % WC;
      const int rest = e / WC;
      g8 = rest % (KC / 8);
      hl = rest / (KC / 8);
    };
    auto load = [&](int s, QuadIn<NSUB, GENQ, v8, CPY>& in) {
      const int c = sm.chunk(s);
      load_quad_inputs<NSUB, GENQ>(a, f, sm.bin(s), c * (KC / 2), ptid, NPT, in);
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        int xc, g8, hl;
        copy_item(k, xc, g8, hl);
        const T* src = reinterpret_cast<const T*>(hl ? a.basis_lo : a.basis_hi);
        in.bc[k] = *reinterpret_cast<const v8*>(src + ((size_t)(c * (KC / 8) + g8) * N + xwg + xc) * 8);
      }
    };
    auto store = [&](int s, const QuadIn<NSUB, GENQ, v8, CPY>& in, T* Ab, T* Bb) {
      const int c0q = sm.chunk(s) * (KC / 2);
#pragma unroll
      for (int k = 0; k < GENQ; ++k) {
        const QuadItem it(ptid + k * NPT);
        float vals[NT][4];
        gen_quad<NSUB>(a, zr[k], in, k, c0q + 2 * it.p4 == 0, vals);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          Quad16<T> hi, lo;
#pragma unroll
          for (int j = 0; j < 4; ++j) hi.v[j] = (T)vals[t][j];
          *reinterpret_cast<Quad16<T>*>(Ab + ((t * NH + 0) * 32 + it.r) * RS + 4 * it.p4) = hi;
          if (NH == 2) {
#pragma unroll
            for (int j = 0; j < 4; ++j) lo.v[j] = (T)(vals[t][j] - (float)hi.v[j]);
            *reinterpret_cast<Quad16<T>*>(Ab + ((t * NH + 1) * 32 + it.r) * RS + 4 * it.p4) = lo;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < CPY; ++k) {
        int xc, g8, hl;
        copy_item(k, xc, g8, hl);
        *reinterpret_cast<v8*>(Bb + (hl * WC + xc) * RS + 8 * g8) = in.bc[k];
      }
    };
    // inputs of stage s+2 are in flight while stage s+1 is generated (ping-pong
    // input sets, as in the FP32 kernel)
    if (S > 0) {
      load(0, cur);
      store(0, cur, Abuf, Bbuf);
    }
    if (S > 1) load(1, cur);
    __syncthreads();
    // Loads are unconditional (the last stage's inputs are re-read past the end) so
    // the in-flight registers never merge with older values at a branch.
    auto step = [&](int s, QuadIn<NSUB, GENQ, v8, CPY>& gen, QuadIn<NSUB, GENQ, v8, CPY>& fill) {
      load(min(s + 2, S - 1), fill);
      store(s + 1, gen, Abuf + ((s + 1) & 1) * A_SZ, Bbuf + ((s + 1) & 1) * B_SZ);
      __syncthreads();
    };
    int s = 0;
    for (; s + 2 < S; s += 2) {
      step(s, cur, nxt);
      step(s + 1, nxt, cur);
    }
    if (s + 1 < S) {
      step(s, cur, nxt);
      ++s;
    }
    if (S > 0) __syncthreads();   // stage S-1: nothing left to generate
    return;
  }

  // ---------------- consumer ----------------
  const int half = lane >> 5, col = lane & 31;
  float accS[1][NSUB][16];
  float accC[1][NP > 0 ? NP : 1][16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[0][i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[0][p][v] = 0.f;
  }
  v16f C[1][NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;

  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const T* Ac = Abuf + (s & 1) * A_SZ;
    const T* Bc = Bbuf + (s & 1) * B_SZ;
#pragma unroll
    for (int ks = 0; ks < KC / 16; ++ks) {
      const int xc = w * 32 + col;
      const v8 bh = *reinterpret_cast<const v8*>(Bc + (0 * WC + xc) * RS + ks * 16 + 8 * half);
      v8 bl;
      if (NH == 2) bl = *reinterpret_cast<const v8*>(Bc + (1 * WC + xc) * RS + ks * 16 + 8 * half);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const v8 ah = *reinterpret_cast<const v8*>(Ac + ((t * NH + 0) * 32 + col) * RS + ks * 16 + 8 * half);
        C[0][t] = Mma<T>::run(ah, bh, C[0][t]);
        if (NH == 2) {
          const v8 al = *reinterpret_cast<const v8*>(Ac + ((t * NH + 1) * 32 + col) * RS + ks * 16 + 8 * half);
          C[0][t] = Mma<T>::run(ah, bl, C[0][t]);
          C[0][t] = Mma<T>::run(al, bh, C[0][t]);
        }
      }
    }
    if (sm.chunk(s) == sm.nch - 1) {
      fold_bin<NSUB, 1>(C, a.inv_scale[(size_t)f * a.n_sel + sm.bin(s)], accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc<NSUB, 1>(a, sp, f, d0, xwg + w * 32, lane, accS, accC);
}

// LDS bytes of the kernels above (double-buffered A and basis tiles)
template <int NSUB, int NC>
constexpr size_t k3_fp32_lds() {
  return (size_t)2 * (2 * NSUB * 32 * 32 + 32 * NC * 32) * sizeof(float);
}
template <int PASSES, int NSUB, int NC>
constexpr size_t k3_split_lds() {
  return (size_t)2 * ((2 * NSUB) * (PASSES == 3 ? 2 : 1) * 32 * 40 + (PASSES == 3 ? 2 : 1) * NC * 32 * 40) * 2;
}

}  // namespace pam
