// K3 with fused wave roles: every wave of the workgroup both generates part of
// the next stage's A tile and runs the matrix-core products of the current one.
//
// Same computation as k3_fields.hpp.  A workgroup owns one frame, 32 depths and
// 256 columns (8 waves, one 32x32 output tile each, two waves per SIMD; N = 256
// or 512, i.e. one or two column groups), so
// every generated A element feeds 256 columns.  Only A goes through LDS: each
// wave reads its basis operand for a stage straight from global memory (L2),
// in a layout where a lane's operand values for the stage are contiguous, and
// reloads the registers of a consumed k-step with the next stage's values while
// the remaining products run.  Per stage a wave
//   (1) runs the products of stage s (A from LDS buffer s&1, basis from
//       registers), refilling the basis registers for stage s+1 as it goes,
//   (2) generates its item of stage s+1's A tile into buffer (s+1)&1 from the
//       bin's inputs staged in LDS,
//   (3) at the first stage of a bin, writes the next bin's staged inputs (read
//       from global memory before the products),
//   (4) waits at the stage barrier.
// Generation item of a thread: one slot pair (cos q, sin q) of one depth row,
// 32 rows x 16 pairs per stage.  In the 16-bit A layout ([row][slot], 80-byte
// rows) 32 lanes cover 8 rows x 4 adjacent pairs, so their 4-byte stores hit 32
// distinct banks; in the FP32 layout ([slot][row]) 32 lanes cover 32 rows.
#pragma once
#include "k3_fields16.hpp"

namespace pam {

struct WgX {
  int sp, xg, dt, f, S, b_end;
  StageMap sm;
  __device__ WgX(const K3Args& a, int kc) {
    int bid = blockIdx.x;
    sp = bid % a.n_split; bid /= a.n_split;
    xg = bid % a.n_xg;    bid /= a.n_xg;
    dt = bid % a.n_dt;    bid /= a.n_dt;
    f = bid;
    const int b_begin = sp * a.bins_per_split;
    b_end = min(a.n_sel, b_begin + a.bins_per_split);
    sm = StageMap{b_begin, a.N / kc};
    S = (b_end - b_begin) * sm.nch;
  }
};

// Per-bin generation inputs staged in LDS (double-buffered by bin parity): the
// folded coefficients of the frame's bin, [NSUB][N] float2 (NSUB N / 2 pieces of
// 16 bytes), then its kz / (2 pi) row, [kz_row(N)] doubles (kz_row(N) / 2
// pieces).  Thread p moves pieces p + 512 k, k < NPC (NPC = 1 for N = 256, 2 for
// N = 512).
template <int NPC>
struct BinPiece {
  uint4 v[NPC];
  __device__ __forceinline__ static uint4 piece(const K3Args& a, int nsub, int f, int b, int i) {
    const int n4 = nsub * a.N / 2;
    if (i < n4) return *reinterpret_cast<const uint4*>(a.coeffs + ((size_t)f * a.n_sel + b) * nsub * a.N + 2 * i);
    return *reinterpret_cast<const uint4*>(a.kz + (size_t)b * kz_row(a.N) + 2 * (i - n4));
  }
  __device__ __forceinline__ void load(const K3Args& a, int nsub, int f, int b, int tid) {
    const int np = nsub * a.N / 2 + kz_row(a.N) / 2;
#pragma unroll
    for (int k = 0; k < NPC; ++k)
      if (tid + 512 * k < np) v[k] = piece(a, nsub, f, b, tid + 512 * k);
  }
  // gs: [NSUB N / 2] pieces followed by the kz row
  __device__ __forceinline__ void store(const K3Args& a, int nsub, uint4* gs, int tid) const {
    const int np = nsub * a.N / 2 + kz_row(a.N) / 2;
#pragma unroll
    for (int k = 0; k < NPC; ++k)
      if (tid + 512 * k < np) gs[tid + 512 * k] = v[k];
  }
};

// A values of one slot pair from the staged inputs of its bin:
// vals[t][0..1] = A_t[row, 2q], A_t[row, 2q + 1] for the pair's global q.
template <int NSUB>
__device__ __forceinline__ void x_gen(const K3Args& a, double z, const uint4* gsb, int q,
                                      float vals[2 * NSUB][2]) {
  const float4* gs = reinterpret_cast<const float4*>(gsb);
  const double* ks = reinterpret_cast<const double*>(gsb + NSUB * a.N / 2);
  float2 h0 = make_float2(0.f, 0.f), h1 = h0;
  if (z >= 0.0) {
    h0 = propagator(z, ks[q], a.zero_evanescent);
    h1 = q == 0 ? propagator(z, ks[a.N / 2], a.zero_evanescent) : h0;
  }
#pragma unroll
  for (int i = 0; i < NSUB; ++i) {
    const float4 gg = gs[i * (a.N / 2) + q];
    const float2 a0 = cmul(h0, make_float2(gg.x, gg.y));
    const float2 a1 = cmul(h1, make_float2(gg.z, gg.w));
    vals[2 * i][0] = a0.x;
    vals[2 * i][1] = a1.x;
    vals[2 * i + 1][0] = a0.y;
    vals[2 * i + 1][1] = a1.y;
  }
}

__device__ __forceinline__ uint4 ld16(const void* p) { return *reinterpret_cast<const uint4*>(p); }

// ---------------------------------------------------------------------------
// FP32 operands on v_mfma_f32_32x32x2_f32, KC slots per stage (32 or 64).
// Basis operand layout (basis_lane): [N/32 chunks][N x][2 halves][16], element
// (slot 32 c + 2 j + h, x) at ((c N + x) 2 + h) 16 + j, so lane (x, h) reads the
// values of 4 consecutive k-steps (8 slots) as one 16-byte piece.  The pieces of
// the current and next stage flow through a window of 4 registers: after the
// products of piece g, piece g + 4 (of this stage or the next) is loaded into its
// register.  LDS: A [2][2 NSUB][KC slots][32 rows] floats, then the staged bin
// inputs [2][pieces].  Items of thread p: row p & 31, slot pairs (p >> 5) + 16 k.
// ---------------------------------------------------------------------------
template <int NSUB, int NPC, int KC>
__global__ __launch_bounds__(512, 1) void k3x_fp32(K3Args a) {
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int A_SZ = NT * KC * 32;
  constexpr int NG = KC / 8;     // 16-byte basis pieces per lane per stage
  constexpr int GI = KC / 32;    // generation items per thread per stage
  extern __shared__ float smem[];
  float* Abuf = smem;
  uint4* Gs = reinterpret_cast<uint4*>(smem + 2 * A_SZ);
  const int N = a.N;
  const int GP = NSUB * N / 2 + kz_row(N) / 2;   // staged pieces per bin

  const WgX wg(a, KC);
  const int S = wg.S, f = wg.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d0 = wg.dt * 32;
  const int r = tid & 31;
  const double z = d0 + r < a.n_z ? a.z[d0 + r] : -1.0;
  const int half = lane >> 5, col = lane & 31, xw = w * 32;
  const int xwg = wg.xg * 256;
  const float* bl = a.basis_lane + ((size_t)(xwg + xw + col) * 2 + half) * 16;
  // piece g (0 <= g < NG) of stage s: global 8-slot group G = NG chunk(s) + g
  auto piece = [&](int s, int g) {
    const int G = NG * wg.sm.chunk(s) + g;
    return ld16(bl + (size_t)(G >> 2) * N * 32 + 4 * (G & 3));
  };

  float accS[1][NSUB][16];
  float accC[1][NP > 0 ? NP : 1][16];
  v16f C[1][NT];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[0][i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[0][p][v] = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) C[0][t][v] = 0.f;
  }

  // generation of stage s into buffer s&1 (after the products of the previous stage)
  auto gen = [&](int s) {
    float* Ab = Abuf + (s & 1) * A_SZ;
#pragma unroll
    for (int k = 0; k < GI; ++k) {
      const int ql = (tid >> 5) + 16 * k;
      float vals[NT][2];
      x_gen<NSUB>(a, z, Gs + (wg.sm.bin(s) & 1) * GP, wg.sm.chunk(s) * (KC / 2) + ql, vals);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        Ab[(t * KC + 2 * ql) * 32 + r] = vals[t][0];
        Ab[(t * KC + 2 * ql + 1) * 32 + r] = vals[t][1];
      }
    }
  };
  uint4 bq[4];   // window of basis pieces: piece g lives in bq[g & 3]
  BinPiece<NPC> pc;
  if (S > 0) {
    pc.load(a, NSUB, f, wg.sm.bin(0), tid);
#pragma unroll
    for (int g = 0; g < 4; ++g) bq[g] = g < NG ? piece(0, g) : piece(min(1, S - 1), g - NG);
    pc.store(a, NSUB, Gs + (wg.sm.bin(0) & 1) * GP, tid);
    __syncthreads();
    gen(0);
  }
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const float* Ac = Abuf + (s & 1) * A_SZ;
    const int b = wg.sm.bin(s);
    const bool last = wg.sm.chunk(s) == wg.sm.nch - 1;
    const bool stage_next = wg.sm.chunk(s) == 0 && b + 1 < wg.b_end;
    const float inv = last ? a.inv_scale[(size_t)f * a.n_sel + b] : 0.f;
    if (stage_next) pc.load(a, NSUB, f, b + 1, tid);
    const int sn = min(s + 1, S - 1);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const uint4 pg = bq[g & 3];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = 4 * g + jj;
        const float bv = __uint_as_float(jj == 0 ? pg.x : (jj == 1 ? pg.y : (jj == 2 ? pg.z : pg.w)));
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float av = Ac[(t * KC + 2 * j + half) * 32 + col];
          C[0][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, C[0][t], 0, 0, 0);
        }
      }
      bq[g & 3] = g + 4 < NG ? piece(s, g + 4) : piece(sn, g + 4 - NG);
    }
    if (s + 1 < S) gen(s + 1);
    if (stage_next) pc.store(a, NSUB, Gs + ((b + 1) & 1) * GP, tid);
    if (last) {
      fold_bin<NSUB, 1>(C, inv, accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc<NSUB, 1>(a, wg.sp, f, d0, xwg + xw, lane, accS, accC);
}

// ---------------------------------------------------------------------------
// 16-bit operands on v_mfma_f32_32x32x16_{bf16,f16}, KC slots per stage (32 or 64,
// KC / 16 k-steps).  Basis operand from the slot-group-major 16-bit layout
// ([N/8][N x][8] per plane): lane (x, h) of k-step ks reads group
// (KC / 8) chunk + 2 ks + h; the hi and lo pieces flow through a window of two
// k-steps.  LDS: A [2][2 NSUB][hi, lo][32 rows][KC + 8] 16-bit, then the staged
// bin inputs.  Items of thread p: slot pairs (p & 3) + 4 ((p >> 7) & 3) + 16 k,
// row ((p >> 2) & 7) + 8 ((p >> 5) & 3).
// ---------------------------------------------------------------------------
template <typename T, int PASSES, int NSUB, int NPC, int KC>
__global__ __launch_bounds__(512, 1) void k3x_split(K3Args a) {
  typedef typename Mma<T>::v8 v8;
  constexpr int NT = 2 * NSUB;
  constexpr int NP = AccCount<NSUB>::pairs;
  constexpr int RS = KC + 8;
  constexpr int NH = PASSES == 3 ? 2 : 1;
  constexpr int A_SZ = NT * NH * 32 * RS;
  constexpr int NKS = KC / 16;
  constexpr int GI = KC / 32;
  extern __shared__ float smem[];
  T* Abuf = reinterpret_cast<T*>(smem);
  uint4* Gs = reinterpret_cast<uint4*>(Abuf + 2 * A_SZ);
  const int N = a.N;
  const int GP = NSUB * N / 2 + kz_row(N) / 2;

  const WgX wg(a, KC);
  const int S = wg.S, f = wg.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d0 = wg.dt * 32;
  const int qb = (tid & 3) + 4 * ((tid >> 7) & 3);
  const int rr = ((tid >> 2) & 7) + 8 * ((tid >> 5) & 3);
  const double z = d0 + rr < a.n_z ? a.z[d0 + rr] : -1.0;
  const int half = lane >> 5, col = lane & 31, xw = w * 32;
  const int xwg = wg.xg * 256;
  const T* bhi = reinterpret_cast<const T*>(a.basis_hi) + (size_t)(xwg + xw + col) * 8;
  const T* blo = reinterpret_cast<const T*>(a.basis_lo) + (size_t)(xwg + xw + col) * 8;
  auto goff = [&](int s, int ks) { return (size_t)((KC / 8) * wg.sm.chunk(s) + 2 * ks + half) * N * 8; };

  float accS[1][NSUB][16];
  float accC[1][NP > 0 ? NP : 1][16];
  v16f C[1][NT];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int i = 0; i < NSUB; ++i) accS[0][i][v] = 0.f;
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) accC[0][p][v] = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) C[0][t][v] = 0.f;
  }

  // generation of stage s into buffer s&1.  The two waves of a SIMD (w and w + 4)
  // order their work differently within a stage, one generating before its products
  // and one after, so one wave's VALU work meets the other's matrix-core products.
  const bool gen_first = w >= 4;
  auto gen = [&](int s) {
    T* Ab = Abuf + (s & 1) * A_SZ;
#pragma unroll
    for (int k = 0; k < GI; ++k) {
      const int ql = qb + 16 * k;
      float vals[NT][2];
      x_gen<NSUB>(a, z, Gs + (wg.sm.bin(s) & 1) * GP, wg.sm.chunk(s) * (KC / 2) + ql, vals);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        Pair16<T> hi, lo;
        hi.x = (T)vals[t][0];
        hi.y = (T)vals[t][1];
        *reinterpret_cast<Pair16<T>*>(Ab + ((t * NH + 0) * 32 + rr) * RS + 2 * ql) = hi;
        if (NH == 2) {
          lo.x = (T)(vals[t][0] - (float)hi.x);
          lo.y = (T)(vals[t][1] - (float)hi.y);
          *reinterpret_cast<Pair16<T>*>(Ab + ((t * NH + 1) * 32 + rr) * RS + 2 * ql) = lo;
        }
      }
    }
  };
  // window of basis operands: k-step ks lives in uh/ul[ks & 1]
  uint4 uh[2], ul[2];
  BinPiece<NPC> pc;
  if (S > 0) {
    pc.load(a, NSUB, f, wg.sm.bin(0), tid);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const size_t o = ks < NKS ? goff(0, ks) : goff(min(1, S - 1), ks - NKS);
      uh[ks] = ld16(bhi + o);
      if (NH == 2) ul[ks] = ld16(blo + o);
    }
    pc.store(a, NSUB, Gs + (wg.sm.bin(0) & 1) * GP, tid);
    __syncthreads();
    gen(0);
  }
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const T* Ac = Abuf + (s & 1) * A_SZ;
    const int b = wg.sm.bin(s);
    const bool last = wg.sm.chunk(s) == wg.sm.nch - 1;
    const bool stage_next = wg.sm.chunk(s) == 0 && b + 1 < wg.b_end;
    const float inv = last ? a.inv_scale[(size_t)f * a.n_sel + b] : 0.f;
    if (stage_next) pc.load(a, NSUB, f, b + 1, tid);
    if (gen_first && s + 1 < S) gen(s + 1);
    const int sn = min(s + 1, S - 1);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const v8 bh = __builtin_bit_cast(v8, uh[ks & 1]);
      v8 bl;
      if (NH == 2) bl = __builtin_bit_cast(v8, ul[ks & 1]);
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
      // k-step ks + 2 of this stage or the next
      const size_t o = ks + 2 < NKS ? goff(s, ks + 2) : goff(sn, ks + 2 - NKS);
      uh[ks & 1] = ld16(bhi + o);
      if (NH == 2) ul[ks & 1] = ld16(blo + o);
    }
    if (!gen_first && s + 1 < S) gen(s + 1);
    if (stage_next) pc.store(a, NSUB, Gs + ((b + 1) & 1) * GP, tid);
    if (last) {
      fold_bin<NSUB, 1>(C, inv, accS, accC);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) C[0][t][v] = 0.f;
    }
    __syncthreads();
  }
  store_acc<NSUB, 1>(a, wg.sp, f, d0, xwg + xw, lane, accS, accC);
}

// LDS bytes of the kernels above for lateral size N
template <int NSUB, int KC>
inline size_t k3x_fp32_lds(int N) {
  return (size_t)2 * (2 * NSUB) * KC * 32 * sizeof(float) + (size_t)2 * (NSUB * N / 2 + kz_row(N) / 2) * 16;
}
template <int PASSES, int NSUB, int KC>
inline size_t k3x_split_lds(int N) {
  return (size_t)2 * (2 * NSUB) * (PASSES == 3 ? 2 : 1) * 32 * (KC + 8) * 2 +
         (size_t)2 * (NSUB * N / 2 + kz_row(N) / 2) * 16;
}

}  // namespace pam
