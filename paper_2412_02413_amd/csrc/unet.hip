// HIP kernels of the NCC-mask surrogate network (gfx950): BF16 NHWC activations,
// FP32 master weights and accumulation.  See include/pam_nn.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/pam_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

inline pam_status_t launched() { return hipGetLastError() == hipSuccess ? PAM_OK : PAM_ERR_DEVICE; }

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM on v_mfma_f32_32x32x16_bf16, staged in LDS.
// GEMM: rows = 32 consecutive pixels of one image row, columns = 32 output
// channels, K = 9 taps x k_in channels.  A tile is 4 RW image rows x 32 columns x
// 32 NO output channels; wave w owns its rows RW w .. RW w + RW - 1, i.e. RW x NO
// accumulator tiles of 32 x 32.  Per chunk of 32 input channels the workgroup stages
// in LDS
//   the input patch: (4 RW + 2) rows x 34 columns (one-pixel halo, zeros outside the
//     image) x 32 channels, and
//   the weights: 9 taps x 32 NO output channels x 32 channels,
// each pixel / output channel padded to 40 BF16 (80 bytes) so that the 32 lanes of a
// 16-byte operand read spread over the banks.  All 9 taps then read their A operand
// (pixel shifted by the tap) and B operand from LDS: one A fragment feeds NO
// products and one B fragment RW products.
//
// A workgroup walks a run of tiles (same output-channel group), chunk by chunk.
// While the products of one (tile, chunk) item run, each thread's pieces of the next
// item (16 bytes each) are already loading into registers; they go to LDS between
// the two barriers that close the item.  With a single chunk the weights stay in LDS
// for the whole run.
// ---------------------------------------------------------------------------
struct ConvArgs {
  const bf16* x;
  const bf16* wt;
  const float* bias;
  bf16* y;
  int32_t ldx, batch, h, w, k_in, ldy, n_out, relu, flip, acc;
  int32_t n_rt, n_ct;   // row tiles (4 RW rows) and column tiles (32) per image
  int32_t n_tiles;      // batch n_rt n_ct
  int32_t run;          // tiles per workgroup
};

constexpr int kConvPad = 40;   // BF16 per staged pixel or output channel (32 used)

template <int RW, int NO>
constexpr int conv_lds_bytes() {
  return ((4 * RW + 2) * 34 + 9 * 32 * NO) * kConvPad * 2;
}

template <int RW, int NO>
__global__ __launch_bounds__(256, 2) void conv3x3_kernel(ConvArgs a) {
  constexpr int PR = 4 * RW + 2;                 // patch rows
  constexpr int CO = 32 * NO;                    // output channels per workgroup
  constexpr int NIN = PR * 34 * 4;               // 16-byte input pieces per chunk
  constexpr int NW = 9 * CO * 4;                 // 16-byte weight pieces per chunk
  constexpr int PIN = (NIN + 255) / 256;         // per thread
  constexpr int PW = (NW + 255) / 256;
  extern __shared__ __align__(16) bf16 lds_c[];
  bf16* xin = lds_c;                             // [PR][34][kConvPad]
  bf16* wts = lds_c + PR * 34 * kConvPad;        // [9][CO][kConvPad]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = lane & 31, half = lane >> 5;
  const int co0 = blockIdx.y * CO;
  const int nch = a.k_in / 32;
  const int t_begin = blockIdx.x * a.run;
  const int t_end = min(a.n_tiles, t_begin + a.run);
  const int n_items = (t_end - t_begin) * nch;
  const v8bf zero = {};

  v8bf pin[PIN], pw[PW];
  // registers <- pieces of item `it` (tile t_begin + it / nch, chunk it % nch)
  auto fetch = [&](int it, bool with_w) {
    const int tile = t_begin + it / nch, k0 = 32 * (it % nch);
    const int ct = tile % a.n_ct, rt = (tile / a.n_ct) % a.n_rt, img = tile / (a.n_ct * a.n_rt);
    const int r0 = rt * 4 * RW, c0 = ct * 32;
#pragma unroll
    for (int j = 0; j < PIN; ++j) {
      const int e = tid + 256 * j;
      const int q = e & 3, pc = (e >> 2) % 34, pr = (e >> 2) / 34;
      const int row = r0 - 1 + pr, col = c0 - 1 + pc;
      pin[j] = zero;
      if (e < NIN && row >= 0 && row < a.h && col >= 0 && col < a.w)
        pin[j] = *reinterpret_cast<const v8bf*>(a.x + (((int64_t)img * a.h + row) * a.w + col) * (int64_t)a.ldx +
                                                k0 + 8 * q);
    }
    if (with_w) {
#pragma unroll
      for (int j = 0; j < PW; ++j) {
        const int e = tid + 256 * j;
        const int q = e & 3, t = (e >> 2) % 9, o = (e >> 2) / 9;
        if (e < NW) pw[j] = *reinterpret_cast<const v8bf*>(a.wt + ((int64_t)(co0 + o) * 9 + t) * a.k_in + k0 + 8 * q);
      }
    }
  };
  auto put = [&](bool with_w) {
#pragma unroll
    for (int j = 0; j < PIN; ++j) {
      const int e = tid + 256 * j;
      const int q = e & 3, pc = (e >> 2) % 34, pr = (e >> 2) / 34;
      if (e < NIN) *reinterpret_cast<v8bf*>(xin + (pr * 34 + pc) * kConvPad + 8 * q) = pin[j];
    }
    if (with_w) {
#pragma unroll
      for (int j = 0; j < PW; ++j) {
        const int e = tid + 256 * j;
        const int q = e & 3, t = (e >> 2) % 9, o = (e >> 2) / 9;
        if (e < NW) *reinterpret_cast<v8bf*>(wts + (t * CO + o) * kConvPad + 8 * q) = pw[j];
      }
    }
  };

  v16f C[RW][NO];
  auto clear = [&]() {
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int n = 0; n < NO; ++n)
#pragma unroll
        for (int v = 0; v < 16; ++v) C[r][n][v] = 0.f;
  };
  clear();
  if (n_items > 0) fetch(0, true);
  for (int it = 0; it < n_items; ++it) {
    const bool w_now = nch > 1 || it == 0;       // weights of this item go to LDS
    put(w_now);
    __syncthreads();
    if (it + 1 < n_items) fetch(it + 1, nch > 1);
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
      int dh = t / 3 - 1, dw = t % 3 - 1;
      if (a.flip) {
        dh = -dh;
        dw = -dw;
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        v8bf av[RW], bv[NO];
#pragma unroll
        for (int r = 0; r < RW; ++r)
          av[r] = *reinterpret_cast<const v8bf*>(xin + ((RW * wv + r + 1 + dh) * 34 + i + 1 + dw) * kConvPad + 16 * ks +
                                                 8 * half);
#pragma unroll
        for (int n = 0; n < NO; ++n)
          bv[n] = *reinterpret_cast<const v8bf*>(wts + (t * CO + 32 * n + i) * kConvPad + 16 * ks + 8 * half);
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int n = 0; n < NO; ++n) C[r][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[r], bv[n], C[r][n], 0, 0, 0);
      }
    }
    __syncthreads();
    if (it % nch == nch - 1) {
      // last chunk of the tile: bias / activation / accumulation and store
      const int tile = t_begin + it / nch;
      const int ct = tile % a.n_ct, rt = (tile / a.n_ct) % a.n_rt, img = tile / (a.n_ct * a.n_rt);
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = rt * 4 * RW + RW * wv + r;
        if (row >= a.h) continue;
        const int64_t p0 = ((int64_t)img * a.h + row) * a.w + ct * 32;
#pragma unroll
        for (int n = 0; n < NO; ++n) {
          const int co = co0 + 32 * n + i;
          const float bb = (a.bias && !a.acc) ? a.bias[co] : 0.f;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int px = 8 * (v >> 2) + 4 * half + (v & 3);
            bf16* dst = a.y + (p0 + px) * (int64_t)a.ldy + co;
            float val = C[r][n][v] + bb;
            if (a.acc) {
              val += (float)*dst;
            } else if (a.relu) {
              val = fmaxf(val, 0.f);
            }
            *dst = (bf16)val;
          }
        }
      }
      clear();
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient on v_mfma_f32_32x32x16_bf16: dW[t] = X_t^T dY, a GEMM whose K runs
// over pixels.  One workgroup per (32 input channels, 32 output channels, tap, pixel
// chunk).  Per slab of 256 pixels the workgroup stages x (shifted by the tap; zeros
// outside the image and past the chunk) and dy in LDS transposed, [32 channels][256
// pixels + 8] BF16, so that an operand fragment (8 consecutive pixels of one channel)
// is one 16-byte read.  Wave w takes pixels 64 w .. 64 w + 63 of the slab: four
// products of K = 16 into one 32 x 32 FP32 tile.  At the end the four waves' tiles are
// summed in LDS and each thread adds four values to dW with atomics.  The products of
// two BF16 values are exact in FP32, so only the accumulation order differs from an
// FP32 sum of the same BF16 operands.
// ---------------------------------------------------------------------------
struct WgradArgs {
  const bf16* x;
  const bf16* dy;
  float* dw;
  int64_t P, chunk;
  int32_t ldx, lddy, h, w, c_in, c_out;
};

constexpr int kWgSlab = 256;              // pixels per staged slab
constexpr int kWgPitch = kWgSlab + 8;     // BF16 per staged channel row (16-byte aligned rows)

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ __align__(16) bf16 xt[32 * kWgPitch];
  __shared__ __align__(16) bf16 dt[32 * kWgPitch];
  const int c0 = blockIdx.x * 32, o0 = blockIdx.y * 32;
  const int t = blockIdx.z % 9;
  const int64_t chunk = blockIdx.z / 9;
  const int dh = t / 3 - 1, dw = t % 3 - 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = lane & 31, half = lane >> 5;
  const int q = tid & 3;                  // channels 8 q .. 8 q + 7 of the thread's pieces
  const int64_t pbeg = chunk * a.chunk;
  const int64_t pend = min(a.P, pbeg + a.chunk);
  v16f C;
#pragma unroll
  for (int v = 0; v < 16; ++v) C[v] = 0.f;
  for (int64_t pr = pbeg; pr < pend; pr += kWgSlab) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = (tid >> 2) + 64 * r;   // slab pixel of piece tid + 256 r
      const int64_t p = pr + j;
      v8bf xv = {}, dv = {};
      if (p < pend) {
        const int wc = (int)(p % a.w);
        const int64_t rr = p / a.w;
        const int hr = (int)(rr % a.h);
        const int64_t img = rr / a.h;
        const int hh = hr + dh, ww = wc + dw;
        if (hh >= 0 && hh < a.h && ww >= 0 && ww < a.w)
          xv = *reinterpret_cast<const v8bf*>(a.x + ((img * a.h + hh) * a.w + ww) * (int64_t)a.ldx + c0 + 8 * q);
        dv = *reinterpret_cast<const v8bf*>(a.dy + p * (int64_t)a.lddy + o0 + 8 * q);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        xt[(8 * q + k) * kWgPitch + j] = xv[k];
        dt[(8 * q + k) * kWgPitch + j] = dv[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k0 = 64 * wv + 16 * s + 8 * half;   // A[c = i][k0 .. k0 + 7], B[k0 .. k0 + 7][o = i]
      const v8bf av = *reinterpret_cast<const v8bf*>(xt + i * kWgPitch + k0);
      const v8bf bv = *reinterpret_cast<const v8bf*>(dt + i * kWgPitch + k0);
      C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, C, 0, 0, 0);
    }
    __syncthreads();
  }
  // C[v] holds (c = 8 (v / 4) + 4 half + v % 4, o = i); the waves' tiles meet in LDS
  // (16 KiB in xt, free since the last barrier)
  float* red = reinterpret_cast<float*>(xt);         // [4 waves][32 c][32 o]
#pragma unroll
  for (int v = 0; v < 16; ++v) red[(wv * 32 + 8 * (v >> 2) + 4 * half + (v & 3)) * 32 + i] = C[v];
  __syncthreads();
  for (int e = tid; e < 1024; e += 256) {
    const float sum = red[e] + red[1024 + e] + red[2048 + e] + red[3072 + e];
    atomicAdd(a.dw + ((int64_t)t * a.c_in + c0 + (e >> 5)) * a.c_out + o0 + (e & 31), sum);
  }
}

// column sums of dy over pixels: one workgroup per (channel tile of 64, pixel chunk)
__global__ __launch_bounds__(256) void colsum_kernel(const bf16* dy, int32_t lddy, int64_t P, int32_t c, int64_t chunk,
                                                     float* out) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int ch = blockIdx.x * 64 + cl;
  const int64_t pbeg = (int64_t)blockIdx.y * chunk, pend = min(P, pbeg + chunk);
  float s = 0.f;
  if (ch < c)
    for (int64_t p = pbeg + g; p < pend; p += 4) s += (float)dy[p * lddy + ch];
  red[g][cl] = s;
  __syncthreads();
  if (g == 0 && ch < c) atomicAdd(out + ch, red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl]);
}

__global__ void relu_bwd_kernel(const bf16* y, int32_t ldy, bf16* dy, int32_t lddy, int64_t n, int32_t c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t p = e / c;
  const int k = (int)(e - p * c);
  if (!((float)y[p * ldy + k] > 0.f)) dy[p * lddy + k] = (bf16)0.f;
}

__global__ void maxpool_kernel(const bf16* x, int32_t ldx, int64_t n, int32_t h, int32_t w, int32_t c, bf16* y,
                               int32_t ldy, uint8_t* arg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // n = batch * (h/2) * (w/2) * c
  const int k = (int)(e % c);
  const int64_t q = e / c;
  const int wo = (int)(q % (w / 2));
  const int64_t r = q / (w / 2);
  const int ho = (int)(r % (h / 2));
  const int64_t img = r / (h / 2);
  const int64_t base = (img * h + 2 * ho) * (int64_t)w + 2 * wo;
  const float v[4] = {(float)x[base * ldx + k], (float)x[(base + 1) * ldx + k], (float)x[(base + w) * ldx + k],
                      (float)x[(base + w + 1) * ldx + k]};
  int best = 0;
  for (int j = 1; j < 4; ++j)
    if (v[j] > v[best]) best = j;
  y[q * ldy + k] = (bf16)v[best];
  arg[e] = (uint8_t)best;
}

__global__ void maxpool_bwd_kernel(const bf16* dy, int32_t lddy, const uint8_t* arg, int64_t n, int32_t h, int32_t w,
                                   int32_t c, bf16* dx, int32_t lddx, int32_t accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // n = batch * (h/2) * (w/2) * c
  const int k = (int)(e % c);
  const int64_t q = e / c;
  const int wo = (int)(q % (w / 2));
  const int64_t r = q / (w / 2);
  const int ho = (int)(r % (h / 2));
  const int64_t img = r / (h / 2);
  const int64_t base = (img * h + 2 * ho) * (int64_t)w + 2 * wo;
  const int64_t pos[4] = {base, base + 1, base + w, base + w + 1};
  const float g = (float)dy[q * lddy + k];
  const int best = arg[e];
  for (int j = 0; j < 4; ++j) {
    bf16* d = dx + pos[j] * lddx + k;
    const float add = (j == best) ? g : 0.f;
    *d = (bf16)(accumulate ? (float)*d + add : add);
  }
}

__global__ void upsample_kernel(const bf16* x, int32_t ldx, int64_t n, int32_t h, int32_t w, int32_t c, bf16* y,
                                int32_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // n = batch * (2h) * (2w) * c
  const int k = (int)(e % c);
  const int64_t q = e / c;
  const int wo = (int)(q % (2 * w));
  const int64_t r = q / (2 * w);
  const int ho = (int)(r % (2 * h));
  const int64_t img = r / (2 * h);
  y[q * ldy + k] = x[((img * h + ho / 2) * w + wo / 2) * (int64_t)ldx + k];
}

__global__ void upsample_bwd_kernel(const bf16* dy, int32_t lddy, int64_t n, int32_t h, int32_t w, int32_t c, bf16* dx,
                                    int32_t lddx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // n = batch * h * w * c (sizes of dx)
  const int k = (int)(e % c);
  const int64_t q = e / c;
  const int wc = (int)(q % w);
  const int64_t r = q / w;
  const int hr = (int)(r % h);
  const int64_t img = r / h;
  const int64_t base = (img * 2 * h + 2 * hr) * (int64_t)(2 * w) + 2 * wc;
  const float s = (float)dy[base * lddy + k] + (float)dy[(base + 1) * lddy + k] +
                  (float)dy[(base + 2 * w) * lddy + k] + (float)dy[(base + 2 * w + 1) * lddy + k];
  dx[q * lddx + k] = (bf16)s;
}

__device__ __forceinline__ float sigmoidf_(float z) { return 1.f / (1.f + expf(-z)); }
__device__ __forceinline__ float softplusf_(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }

// The same four operations on 8 channels (16 bytes) per thread, for channel counts and
// strides that are multiples of 8 on 16-byte aligned tensors (every tensor of the network).
__global__ void maxpool8_kernel(const bf16* x, int32_t ldx, int64_t n8, int32_t h, int32_t w, int32_t c8, bf16* y,
                                int32_t ldy, uint8_t* arg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n8) return;  // n8 = batch * (h/2) * (w/2) * c/8
  const int k = (int)(e % c8) * 8;
  const int64_t q = e / c8;
  const int wo = (int)(q % (w / 2));
  const int64_t r = q / (w / 2);
  const int ho = (int)(r % (h / 2));
  const int64_t img = r / (h / 2);
  const int64_t base = (img * h + 2 * ho) * (int64_t)w + 2 * wo;
  const v8bf v[4] = {*reinterpret_cast<const v8bf*>(x + base * ldx + k),
                     *reinterpret_cast<const v8bf*>(x + (base + 1) * ldx + k),
                     *reinterpret_cast<const v8bf*>(x + (base + w) * ldx + k),
                     *reinterpret_cast<const v8bf*>(x + (base + w + 1) * ldx + k)};
  v8bf out;
  uint64_t bests = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int best = 0;
    float bv = (float)v[0][j];
#pragma unroll
    for (int m = 1; m < 4; ++m)
      if ((float)v[m][j] > bv) {
        bv = (float)v[m][j];
        best = m;
      }
    out[j] = v[best][j];
    bests |= (uint64_t)best << (8 * j);
  }
  *reinterpret_cast<v8bf*>(y + q * ldy + k) = out;
  *reinterpret_cast<uint64_t*>(arg + e * 8) = bests;
}

__global__ void maxpool8_bwd_kernel(const bf16* dy, int32_t lddy, const uint8_t* arg, int64_t n8, int32_t h,
                                    int32_t w, int32_t c8, bf16* dx, int32_t lddx, int32_t accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n8) return;
  const int k = (int)(e % c8) * 8;
  const int64_t q = e / c8;
  const int wo = (int)(q % (w / 2));
  const int64_t r = q / (w / 2);
  const int ho = (int)(r % (h / 2));
  const int64_t img = r / (h / 2);
  const int64_t base = (img * h + 2 * ho) * (int64_t)w + 2 * wo;
  const int64_t pos[4] = {base, base + 1, base + w, base + w + 1};
  const v8bf g = *reinterpret_cast<const v8bf*>(dy + q * lddy + k);
  const uint64_t bests = *reinterpret_cast<const uint64_t*>(arg + e * 8);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v8bf* d = reinterpret_cast<v8bf*>(dx + pos[m] * lddx + k);
    const v8bf old = accumulate ? *d : v8bf{};
    v8bf o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float add = (int)((bests >> (8 * j)) & 0xff) == m ? (float)g[j] : 0.f;
      o[j] = (bf16)(accumulate ? (float)old[j] + add : add);
    }
    *d = o;
  }
}

__global__ void upsample8_kernel(const bf16* x, int32_t ldx, int64_t n8, int32_t h, int32_t w, int32_t c8, bf16* y,
                                 int32_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n8) return;  // n8 = batch * (2h) * (2w) * c/8
  const int k = (int)(e % c8) * 8;
  const int64_t q = e / c8;
  const int wo = (int)(q % (2 * w));
  const int64_t r = q / (2 * w);
  const int ho = (int)(r % (2 * h));
  const int64_t img = r / (2 * h);
  *reinterpret_cast<v8bf*>(y + q * ldy + k) =
      *reinterpret_cast<const v8bf*>(x + ((img * h + ho / 2) * w + wo / 2) * (int64_t)ldx + k);
}

__global__ void upsample8_bwd_kernel(const bf16* dy, int32_t lddy, int64_t n8, int32_t h, int32_t w, int32_t c8,
                                     bf16* dx, int32_t lddx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n8) return;  // n8 = batch * h * w * c/8 (sizes of dx)
  const int k = (int)(e % c8) * 8;
  const int64_t q = e / c8;
  const int wc = (int)(q % w);
  const int64_t r = q / w;
  const int hr = (int)(r % h);
  const int64_t img = r / h;
  const int64_t base = (img * 2 * h + 2 * hr) * (int64_t)(2 * w) + 2 * wc;
  const v8bf a = *reinterpret_cast<const v8bf*>(dy + base * lddy + k);
  const v8bf b = *reinterpret_cast<const v8bf*>(dy + (base + 1) * lddy + k);
  const v8bf c = *reinterpret_cast<const v8bf*>(dy + (base + 2 * w) * lddy + k);
  const v8bf d = *reinterpret_cast<const v8bf*>(dy + (base + 2 * w + 1) * lddy + k);
  v8bf o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = (bf16)((float)a[j] + (float)b[j] + (float)c[j] + (float)d[j]);
  *reinterpret_cast<v8bf*>(dx + q * lddx + k) = o;
}

__global__ __launch_bounds__(256) void head_kernel(const bf16* feat, int32_t c, int64_t P, const float* w,
                                                   const float* b, const float* target, const float* weight,
                                                   float* mask, float* err, float* dz, float* loss,
                                                   float inv_count) {
  __shared__ float red[3][256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float l0 = 0.f, l1 = 0.f, l2 = 0.f;
  if (p < P) {
    float z0 = b[0], z1 = b[1];
    if ((c & 7) == 0) {
      for (int k = 0; k < c; k += 8) {
        const v8bf f8 = *reinterpret_cast<const v8bf*>(feat + p * c + k);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float f = (float)f8[j];
          z0 = fmaf(f, w[2 * (k + j)], z0);
          z1 = fmaf(f, w[2 * (k + j) + 1], z1);
        }
      }
    } else {
      for (int k = 0; k < c; ++k) {
        const float f = (float)feat[p * c + k];
        z0 = fmaf(f, w[2 * k], z0);
        z1 = fmaf(f, w[2 * k + 1], z1);
      }
    }
    const float m = sigmoidf_(z0), e = sigmoidf_(z1);
    mask[p] = m;
    err[p] = e;
    if (target) {
      const float wp = weight ? weight[p] : inv_count;
      const float t = target[p];
      const float ae = fabsf(m - t);
      // binary cross-entropy of sigmoid outputs: t softplus(-z) + (1 - t) softplus(z)
      l0 = wp * (t * softplusf_(-z0) + (1.f - t) * softplusf_(z0));
      l1 = wp * (ae * softplusf_(-z1) + (1.f - ae) * softplusf_(z1));
      l2 = wp * ae;
      if (dz) {
        dz[2 * p] = (m - t) * wp;
        dz[2 * p + 1] = (e - ae) * wp;
      }
    }
  }
  if (!loss) return;  // grid-uniform
  red[0][threadIdx.x] = l0;
  red[1][threadIdx.x] = l1;
  red[2][threadIdx.x] = l2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(loss, red[0][0]);
    atomicAdd(loss + 1, red[1][0]);
    atomicAdd(loss + 2, red[2][0]);
  }
}

// w[f][p] = ((1 - mix) E[f][p] / sum_p E[f][p] + mix / P) / batch
__global__ __launch_bounds__(1024) void loss_weights_kernel(const float* E, int64_t P, float mix, float inv_batch,
                                                            float* out) {
  __shared__ float red[1024];
  const int64_t f = blockIdx.x;
  float s = 0.f;
  for (int64_t p = threadIdx.x; p < P; p += 1024) s += E[f * P + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const float inv = red[0] > 0.f ? (1.f - mix) / red[0] : 0.f;
  const float u = (red[0] > 0.f ? mix : 1.f) / (float)P;
  for (int64_t p = threadIdx.x; p < P; p += 1024) out[f * P + p] = (E[f * P + p] * inv + u) * inv_batch;
}

__global__ void head_dfeat_kernel(int32_t c, int64_t n, const float* w, const float* dz, bf16* dfeat) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;  // n = P * c
  const int64_t p = e / c;
  const int k = (int)(e - p * c);
  dfeat[e] = (bf16)(dz[2 * p] * w[2 * k] + dz[2 * p + 1] * w[2 * k + 1]);
}

// feat^T dz and column sums of dz: one workgroup per pixel chunk; thread k < 2c
// owns dw[k / 2][k % 2], threads 2c, 2c+1 own db.
__global__ __launch_bounds__(256) void head_dw_kernel(const bf16* feat, int32_t c, int64_t P, int64_t chunk,
                                                      const float* dz, float* dw, float* db) {
  const int k = threadIdx.x;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(P, pbeg + chunk);
  if (k >= 2 * c + 2) return;
  float s = 0.f;
  if (k < 2 * c) {
    const int ch = k >> 1, o = k & 1;
    for (int64_t p = pbeg; p < pend; ++p) s = fmaf((float)feat[p * c + ch], dz[2 * p + o], s);
    atomicAdd(dw + k, s);
  } else {
    const int o = k - 2 * c;
    for (int64_t p = pbeg; p < pend; ++p) s += dz[2 * p + o];
    atomicAdd(db + o, s);
  }
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void pack_kernel(const float* w, int32_t ci, int32_t co, bf16* wt, bf16* wd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)9 * ci * co) return;  // e indexes W[t][c][o]
  const int o = (int)(e % co);
  const int64_t q = e / co;
  const int c = (int)(q % ci);
  const int t = (int)(q / ci);
  const bf16 v = (bf16)w[e];
  wt[((int64_t)o * 9 + t) * ci + c] = v;
  if (wd) wd[((int64_t)c * 9 + t) * co + o] = v;
}

__global__ __launch_bounds__(1024) void features_kernel(const float* E, int64_t P, bf16* out) {
  __shared__ float red[1024];
  const int64_t f = blockIdx.x;
  const float* e = E + f * P;
  float m = 0.f;
  for (int64_t p = threadIdx.x; p < P; p += 1024) m = fmaxf(m, e[p]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float mx = red[0] > 0.f ? red[0] : 1.f;
  const float inv = 1.f / mx;
  for (int64_t p = threadIdx.x; p < P; p += 1024) {
    const float r = e[p] * inv;
    const float lg = fminf(fmaxf(log10f(fmaxf(r, 1e-30f)) / 6.f + 1.f, 0.f), 1.f);
    v8bf lo = {}, z = {};
    lo[0] = (bf16)lg;
    lo[1] = (bf16)r;
    v8bf* dst = reinterpret_cast<v8bf*>(out + (f * P + p) * 32);
    dst[0] = lo;
    dst[1] = z;
    dst[2] = z;
    dst[3] = z;
  }
}

// Input features from the adjacent-pixel cross-spectra of a full-aperture field, in
// three launches over (pixel block, frame): clear the per-frame maxima; sum the channels
// over the bin splits into the energy (S) and raise the frame's maximum (S >= 0, so its
// bit pattern orders like the value: an integer atomic max); write the eight feature
// channels of every pixel.  A pair's normalised cross-spectrum is taken at its even
// member (left column, upper depth), so both pixels of a pair see the same oriented value.
__global__ void clear_max_kernel(unsigned* fmax, int32_t n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) fmax[k] = 0u;
}

// A workgroup covers kEnergyPix pixels of one frame (16 per thread), so a frame's maximum
// takes a few dozen atomics on its address rather than one per 256 pixels: same-address
// atomics are serialised in L2.
constexpr int kEnergyPix = 256 * 16;
__global__ __launch_bounds__(256) void energy_max_kernel(const float* acc, int32_t n_split, int64_t sstride,
                                                         int64_t P, float* energy, unsigned* fmax) {
  __shared__ float red[256];
  const int64_t f = blockIdx.y;
  const int64_t p0 = (int64_t)blockIdx.x * kEnergyPix + threadIdx.x;
  float v = 0.f;
  for (int k = 0; k < 16; ++k) {
    const int64_t p = p0 + 256 * k;
    if (p < P) {
      const float* a0 = acc + f * 5 * P + p;
      float e = 0.f;
      for (int s = 0; s < n_split; ++s) e += a0[s * sstride];
      e = fmaxf(e, 0.f);
      energy[f * P + p] = e;
      v = fmaxf(v, e);
    }
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(fmax + f, __float_as_uint(red[0]));
}

__global__ __launch_bounds__(256) void coherence_features_kernel(const float* acc, int32_t n_split, int64_t sstride,
                                                                 int32_t n_z, int32_t n_x, const float* energy,
                                                                 const unsigned* fmax, bf16* out) {
  const int64_t f = blockIdx.y;
  const int64_t P = (int64_t)n_z * n_x;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const float* a0 = acc + f * 5 * P;
  const float* e = energy + f * P;
  auto chan = [&](int c, int64_t q) {
    float v = 0.f;
    for (int s = 0; s < n_split; ++s) v += a0[s * sstride + c * P + q];
    return v;
  };
  const float mx = __uint_as_float(fmax[f]);
  const float inv = mx > 0.f ? 1.f / mx : 1.f;
  auto coh = [&](int64_t q0, int64_t q1, int c, float* o) {   // |c|, Re c, Im c of the pair (q0, q1)
    const float d = e[q0] * e[q1];
    if (!(d > 0.f)) {
      o[0] = o[1] = o[2] = 0.f;
      return;
    }
    const float r = rsqrtf(d);
    const float re = fminf(fmaxf(chan(c, q0) * r, -1.f), 1.f), im = fminf(fmaxf(chan(c + 1, q0) * r, -1.f), 1.f);
    o[0] = fminf(sqrtf(re * re + im * im), 1.f);
    o[1] = re;
    o[2] = im;
  };
  const int x = (int)(p % n_x), z = (int)(p / n_x);
  const float r = e[p] * inv;
  float cx[3], cz[3];
  coh((int64_t)z * n_x + (x & ~1), (int64_t)z * n_x + (x | 1), 1, cx);
  coh((int64_t)(z & ~1) * n_x + x, (int64_t)(z | 1) * n_x + x, 3, cz);
  v8bf lo, z8 = {};
  lo[0] = (bf16)fminf(fmaxf(log10f(fmaxf(r, 1e-30f)) / 6.f + 1.f, 0.f), 1.f);
  lo[1] = (bf16)r;
  lo[2] = (bf16)cx[0];
  lo[3] = (bf16)cx[1];
  lo[4] = (bf16)cx[2];
  lo[5] = (bf16)cz[0];
  lo[6] = (bf16)cz[1];
  lo[7] = (bf16)cz[2];
  v8bf* dst = reinterpret_cast<v8bf*>(out + (f * P + p) * 32);
  dst[0] = lo;
  dst[1] = z8;
  dst[2] = z8;
  dst[3] = z8;
}

// Predicted relative L2 error of a frame's image: with the image mask^2 E and a mask
// off by err per pixel, the image error is about 2 mask err E, so
// est = ||2 mask err E|| / ||mask^2 E|| (sums in FP64).
__global__ __launch_bounds__(1024) void error_estimate_kernel(const float* mask, const float* err, const float* E,
                                                              int64_t P, float* est) {
  __shared__ double s0[1024], s1[1024];
  const int64_t f = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += 1024) {
    const double m = mask[f * P + p], e = E[f * P + p];
    const double d = 2.0 * m * (double)err[f * P + p] * e, i = m * m * e;
    a += d * d;
    b += i * i;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) est[f] = s1[0] > 0.0 ? (float)sqrt(s0[0] / s1[0]) : INFINITY;
}

// per-frame confidence: 1 - sum_p E[p] err[p] / sum_p E[p]
__global__ __launch_bounds__(1024) void confidence_kernel(const float* err, const float* E, int64_t P, float* conf) {
  __shared__ float s0[1024], s1[1024];
  const int64_t f = blockIdx.x;
  float a = 0.f, b = 0.f;
  for (int64_t p = threadIdx.x; p < P; p += 1024) {
    const float e = E[f * P + p];
    a = fmaf(e, err[f * P + p], a);
    b += e;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) conf[f] = s1[0] > 0.f ? 1.f - s0[0] / s1[0] : 0.f;
}

// image = mask^2 * E (Eq. 11 with the predicted NNCC)
__global__ void apply_mask_kernel(const float* mask, const float* E, float* image, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) image[i] = mask[i] * mask[i] * E[i];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
// 8-channel vector form applies: channel count and strides multiples of 8, 16-byte aligned bases
inline bool vec8(int c, int ld_a, int ld_b, const void* a, const void* b) {
  return c % 8 == 0 && ld_a % 8 == 0 && ld_b % 8 == 0 && aligned16(a) && aligned16(b);
}

}  // namespace

extern "C" {

pam_status_t pam_nn_conv3x3(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t k_in,
                            const void* wt, const float* bias, void* y, int32_t ldy, int32_t n_out, int32_t relu,
                            int32_t flip, int32_t accumulate, void* hip_stream) {
  if (!x || !wt || !y || batch < 1 || h < 1 || w < 32 || w % 32 || k_in < 32 || k_in % 32 || n_out < 32 ||
      n_out % 32 || ldx < k_in || ldx % 8 || ldy < n_out || !aligned16(x) || !aligned16(wt))
    return PAM_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ConvArgs a{static_cast<const bf16*>(x), static_cast<const bf16*>(wt), bias, static_cast<bf16*>(y), ldx, batch, h,
             w, k_in, ldy, n_out, relu, flip, accumulate, 0, w / 32, 0, 1};
  // 64 output channels x 8 rows per tile where the channels allow, else 32 x 16; runs of
  // up to 8 tiles per workgroup, as long as about 512 workgroups (two per CU, the LDS
  // limit) remain
  const bool wide = n_out % 64 == 0;
  const int rows = wide ? 8 : 16, groups = n_out / (wide ? 64 : 32);
  a.n_rt = (h + rows - 1) / rows;
  const int64_t tiles = (int64_t)batch * a.n_rt * a.n_ct;
  if (tiles > 0x7fffffffLL) return PAM_ERR_INVALID_ARG;
  a.n_tiles = (int)tiles;
  a.run = (int)std::max<int64_t>(1, std::min<int64_t>(8, tiles * groups / 512));
  const dim3 grid((unsigned)((tiles + a.run - 1) / a.run), groups);
  // (more than 64 KB of LDS: the kernel attribute is set before each launch)
  if (wide) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(conv3x3_kernel<2, 2>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<2, 2>()) != hipSuccess)
      return PAM_ERR_DEVICE;
    hipLaunchKernelGGL((conv3x3_kernel<2, 2>), grid, dim3(256), (conv_lds_bytes<2, 2>()), st, a);
  } else {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(conv3x3_kernel<4, 1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<4, 1>()) != hipSuccess)
      return PAM_ERR_DEVICE;
    hipLaunchKernelGGL((conv3x3_kernel<4, 1>), grid, dim3(256), (conv_lds_bytes<4, 1>()), st, a);
  }
  return launched();
}

pam_status_t pam_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy, int32_t batch, int32_t h,
                                  int32_t w, int32_t c_in, int32_t c_out, float* dw, float* db, void* hip_stream) {
  if (!x || !dy || !dw || batch < 1 || h < 1 || w < 1 || c_in < 32 || c_in % 32 || c_out < 32 || c_out % 32 ||
      ldx < c_in || ldx % 8 || lddy < c_out || lddy % 8 || !aligned16(x) || !aligned16(dy))
    return PAM_ERR_INVALID_ARG;
  const int64_t P = (int64_t)batch * h * w;
  const int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(64, P / 4096));
  const int64_t chunk = ((P + n_chunks - 1) / n_chunks + kWgSlab - 1) / kWgSlab * kWgSlab;
  WgradArgs a{static_cast<const bf16*>(x), static_cast<const bf16*>(dy), dw, P, chunk, ldx, lddy, h, w, c_in, c_out};
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(wgrad_kernel, dim3(c_in / 32, c_out / 32, 9 * blocks_for(P, (int)chunk)), dim3(256), 0, st, a);
  if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
  if (db) {
    const int64_t cchunk = 2048;
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(c_out, 64), blocks_for(P, (int)cchunk)), dim3(256), 0, st,
                       static_cast<const bf16*>(dy), lddy, P, c_out, cchunk, db);
  }
  return launched();
}

pam_status_t pam_nn_relu_backward(const void* y, int32_t ldy, void* dy, int32_t lddy, int64_t pixels, int32_t c,
                                  void* hip_stream) {
  if (!y || !dy || pixels < 1 || c < 1 || ldy < c || lddy < c) return PAM_ERR_INVALID_ARG;
  const int64_t n = pixels * c;
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const bf16*>(y), ldy, static_cast<bf16*>(dy), lddy, n, c);
  return launched();
}

pam_status_t pam_nn_maxpool(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t c, void* y,
                            int32_t ldy, uint8_t* arg, void* hip_stream) {
  if (!x || !y || !arg || batch < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1 || ldx < c || ldy < c)
    return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * (h / 2) * (w / 2) * c;
  if (vec8(c, ldx, ldy, x, y) && (reinterpret_cast<uintptr_t>(arg) & 7u) == 0)
    hipLaunchKernelGGL(maxpool8_kernel, dim3(blocks_for(n / 8, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(x), ldx, n / 8, h, w, c / 8,
                       static_cast<bf16*>(y), ldy, arg);
  else
    hipLaunchKernelGGL(maxpool_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const bf16*>(x), ldx, n, h, w, c, static_cast<bf16*>(y), ldy, arg);
  return launched();
}

pam_status_t pam_nn_maxpool_backward(const void* dy, int32_t lddy, const uint8_t* arg, int32_t batch, int32_t h,
                                     int32_t w, int32_t c, void* dx, int32_t lddx, int32_t accumulate,
                                     void* hip_stream) {
  if (!dy || !arg || !dx || batch < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1 || lddy < c || lddx < c)
    return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * (h / 2) * (w / 2) * c;
  if (vec8(c, lddy, lddx, dy, dx) && (reinterpret_cast<uintptr_t>(arg) & 7u) == 0)
    hipLaunchKernelGGL(maxpool8_bwd_kernel, dim3(blocks_for(n / 8, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(dy), lddy, arg, n / 8, h, w,
                       c / 8, static_cast<bf16*>(dx), lddx, accumulate);
  else
    hipLaunchKernelGGL(maxpool_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(dy), lddy, arg, n, h, w, c,
                       static_cast<bf16*>(dx), lddx, accumulate);
  return launched();
}

pam_status_t pam_nn_upsample(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t c, void* y,
                             int32_t ldy, void* hip_stream) {
  if (!x || !y || batch < 1 || h < 1 || w < 1 || c < 1 || ldx < c || ldy < c) return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * 4 * h * w * c;
  if (vec8(c, ldx, ldy, x, y))
    hipLaunchKernelGGL(upsample8_kernel, dim3(blocks_for(n / 8, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(x), ldx, n / 8, h, w, c / 8,
                       static_cast<bf16*>(y), ldy);
  else
    hipLaunchKernelGGL(upsample_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const bf16*>(x), ldx, n, h, w, c, static_cast<bf16*>(y), ldy);
  return launched();
}

pam_status_t pam_nn_upsample_backward(const void* dy, int32_t lddy, int32_t batch, int32_t h, int32_t w, int32_t c,
                                      void* dx, int32_t lddx, void* hip_stream) {
  if (!dy || !dx || batch < 1 || h < 1 || w < 1 || c < 1 || lddy < c || lddx < c) return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * h * w * c;
  if (vec8(c, lddy, lddx, dy, dx))
    hipLaunchKernelGGL(upsample8_bwd_kernel, dim3(blocks_for(n / 8, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(dy), lddy, n / 8, h, w, c / 8,
                       static_cast<bf16*>(dx), lddx);
  else
    hipLaunchKernelGGL(upsample_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(dy), lddy, n, h, w, c,
                       static_cast<bf16*>(dx), lddx);
  return launched();
}

pam_status_t pam_nn_head(const void* feat, int32_t c, int64_t pixels, const float* w, const float* b,
                         const float* target, const float* weight, float* mask, float* err, float* dz, float* loss,
                         int64_t count, void* hip_stream) {
  if (!feat || !w || !b || !mask || !err || c < 1 || pixels < 1 || count < 1 || ((dz || loss) && !target))
    return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(head_kernel, dim3(blocks_for(pixels, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const bf16*>(feat), c, pixels, w, b, target, weight, mask, err, dz, loss,
                     1.0f / (float)count);
  return launched();
}

pam_status_t pam_nn_loss_weights(const float* energy, int32_t batch, int64_t pixels, float mix, float* out,
                                 void* hip_stream) {
  if (!energy || !out || batch < 1 || pixels < 1 || !(mix >= 0.f && mix <= 1.f)) return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(loss_weights_kernel, dim3(batch), dim3(1024), 0, static_cast<hipStream_t>(hip_stream), energy,
                     pixels, mix, 1.0f / (float)batch, out);
  return launched();
}

pam_status_t pam_nn_head_backward(const void* feat, int32_t c, int64_t pixels, const float* w, const float* dz,
                                  void* dfeat, float* dw, float* db, void* hip_stream) {
  if (!feat || !w || !dz || !dfeat || !dw || !db || c < 1 || 2 * c + 2 > 256 || pixels < 1)
    return PAM_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t n = pixels * c;
  hipLaunchKernelGGL(head_dfeat_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, c, n, w, dz,
                     static_cast<bf16*>(dfeat));
  if (hipGetLastError() != hipSuccess) return PAM_ERR_DEVICE;
  const int64_t chunk = 1024;
  hipLaunchKernelGGL(head_dw_kernel, dim3(blocks_for(pixels, (int)chunk)), dim3(256), 0, st,
                     static_cast<const bf16*>(feat), c, pixels, chunk, dz, dw, db);
  return launched();
}

pam_status_t pam_nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                         float eps, int32_t step, void* hip_stream) {
  if (!p || !g || !m || !v || n < 1 || step < 1) return PAM_ERR_INVALID_ARG;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), p, g,
                     m, v, n, lr, beta1, beta2, eps, c1, c2);
  return launched();
}

pam_status_t pam_nn_pack_weights(const float* w, int32_t c_in, int32_t c_out, void* wt, void* wd, void* hip_stream) {
  if (!w || !wt || c_in < 1 || c_out < 1) return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)9 * c_in * c_out;
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), w, c_in,
                     c_out, static_cast<bf16*>(wt), static_cast<bf16*>(wd));
  return launched();
}

pam_status_t pam_nn_features(const float* energy, int32_t batch, int64_t pixels, void* out, void* hip_stream) {
  if (!energy || !out || batch < 1 || pixels < 1 || !aligned16(out)) return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(features_kernel, dim3(batch), dim3(1024), 0, static_cast<hipStream_t>(hip_stream), energy, pixels,
                     static_cast<bf16*>(out));
  return launched();
}

pam_status_t pam_nn_coherence_features(const float* accum, int32_t n_split, int64_t split_stride, int32_t batch,
                                       int32_t n_z, int32_t n_x, void* out, float* energy, float* frame_max,
                                       void* hip_stream) {
  if (!accum || !out || !energy || !frame_max || n_split < 1 || batch < 1 || batch > 65535 || n_z < 2 || n_x < 2 ||
      (n_z & 1) || (n_x & 1) || (n_split > 1 && split_stride < (int64_t)batch * 5 * n_z * n_x) || !aligned16(out))
    return PAM_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t P = (int64_t)n_z * n_x;
  unsigned* fm = reinterpret_cast<unsigned*>(frame_max);
  const dim3 grid(blocks_for(P, 256), batch);
  hipLaunchKernelGGL(clear_max_kernel, dim3(blocks_for(batch, 256)), dim3(256), 0, st, fm, batch);
  hipLaunchKernelGGL(energy_max_kernel, dim3(blocks_for(P, kEnergyPix), batch), dim3(256), 0, st, accum, n_split,
                     split_stride, P, energy, fm);
  hipLaunchKernelGGL(coherence_features_kernel, grid, dim3(256), 0, st, accum, n_split, split_stride, n_z, n_x,
                     energy, fm, static_cast<bf16*>(out));
  return launched();
}

pam_status_t pam_nn_error_estimate(const float* mask, const float* err, const float* energy, int32_t batch,
                                   int64_t pixels, float* est, void* hip_stream) {
  if (!mask || !err || !energy || !est || batch < 1 || pixels < 1) return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(error_estimate_kernel, dim3(batch), dim3(1024), 0, static_cast<hipStream_t>(hip_stream), mask, err,
                     energy, pixels, est);
  return launched();
}

pam_status_t pam_nn_confidence(const float* err, const float* energy, int32_t batch, int64_t pixels, float* conf,
                               void* hip_stream) {
  if (!err || !energy || !conf || batch < 1 || pixels < 1) return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(confidence_kernel, dim3(batch), dim3(1024), 0, static_cast<hipStream_t>(hip_stream), err, energy,
                     pixels, conf);
  return launched();
}

pam_status_t pam_nn_apply_mask(const float* mask, const float* energy, float* image, int64_t n, void* hip_stream) {
  if (!mask || !energy || !image || n < 1) return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(apply_mask_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     mask, energy, image, n);
  return launched();
}

}  // extern "C"
