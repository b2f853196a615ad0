// HIP kernels of the NCC-mask surrogate network (gfx950): BF16 NHWC activations,
// FP32 master weights and accumulation.  See include/pam_nn.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/pam_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

inline bool ok_stream(hipError_t e) { return e == hipSuccess; }
inline pam_status_t launched() { return hipGetLastError() == hipSuccess ? PAM_OK : PAM_ERR_DEVICE; }

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM on v_mfma_f32_32x32x16_bf16.
// GEMM: rows = 32 consecutive pixels of one image row, columns = 32 output
// channels, K = 9 taps x k_in channels.  Each lane gathers the 8 channels of
// its pixel (shifted by the tap, zero outside the image) straight from the
// NHWC tensor (16 contiguous bytes) and 8 weights of its output channel from
// the [n_out][9][k_in] layout (16 contiguous bytes).  One wave per 32 pixels x
// 32 NT output channels (each input fragment feeds NT products), four waves
// (four pixel tiles) per workgroup.
// ---------------------------------------------------------------------------
struct ConvArgs {
  const bf16* x;
  const bf16* wt;
  const float* bias;
  bf16* y;
  int64_t P;
  int32_t ldx, h, w, k_in, ldy, n_out, relu, flip, acc;
};

template <int NT>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * 4 + wv;
  const int64_t p0 = tile * 32;
  if (p0 >= a.P) return;  // wave-uniform; the kernel has no barriers
  const int co0 = blockIdx.y * 32 * NT;
  const int i = lane & 31, half = lane >> 5;
  const int64_t p = p0 + i;
  const int wc = (int)(p % a.w);
  const int64_t r = p / a.w;
  const int hr = (int)(r % a.h);
  const int64_t img = r / a.h;
  v16f C[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int v = 0; v < 16; ++v) C[n][v] = 0.f;
  const v8bf zero = {};
  for (int t = 0; t < 9; ++t) {
    int dh = t / 3 - 1, dw = t % 3 - 1;
    if (a.flip) {
      dh = -dh;
      dw = -dw;
    }
    const int hh = hr + dh, ww = wc + dw;
    const bool valid = hh >= 0 && hh < a.h && ww >= 0 && ww < a.w;
    const bf16* xr = a.x + ((img * a.h + (valid ? hh : 0)) * a.w + (valid ? ww : 0)) * (int64_t)a.ldx + 8 * half;
    const bf16* wr = a.wt + ((int64_t)(co0 + i) * 9 + t) * a.k_in + 8 * half;
    const int64_t wstep = (int64_t)32 * 9 * a.k_in;   // next 32 output channels
    // each input fragment feeds NT output tiles
#pragma unroll 2
    for (int k0 = 0; k0 < a.k_in; k0 += 16) {
      const v8bf av = valid ? *reinterpret_cast<const v8bf*>(xr + k0) : zero;
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const v8bf bv = *reinterpret_cast<const v8bf*>(wr + n * wstep + k0);
        C[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, C[n], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int co = co0 + 32 * n + i;
    const float bb = (a.bias && !a.acc) ? a.bias[co] : 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 8 * (v >> 2) + 4 * half + (v & 3);
      bf16* dst = a.y + (p0 + row) * (int64_t)a.ldy + co;
      float val = C[n][v] + bb;
      if (a.acc) {
        val += (float)*dst;
      } else if (a.relu) {
        val = fmaxf(val, 0.f);
      }
      *dst = (bf16)val;
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: one workgroup per (32 input channels, 32 output channels,
// tap, pixel chunk).  Tiles of 64 pixels of x (shifted by the tap) and dy are
// staged in LDS as FP32; each thread accumulates a 2x2 block of (c, o) over the
// chunk and adds it to dW with one atomic per value.
// ---------------------------------------------------------------------------
struct WgradArgs {
  const bf16* x;
  const bf16* dy;
  float* dw;
  int64_t P, chunk;
  int32_t ldx, lddy, h, w, c_in, c_out;
};

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ float xs[64][33];
  __shared__ float ds[64][33];
  const int c0 = blockIdx.x * 32, o0 = blockIdx.y * 32;
  const int t = blockIdx.z % 9;
  const int64_t chunk = blockIdx.z / 9;
  const int dh = t / 3 - 1, dw = t % 3 - 1;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  float acc[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
  const int64_t pbeg = chunk * a.chunk;
  const int64_t pend = min(a.P, pbeg + a.chunk);
  for (int64_t pr = pbeg; pr < pend; pr += 64) {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int j = e >> 5, c = e & 31;
      const int64_t p = pr + j;
      float xv = 0.f, dv = 0.f;
      if (p < pend) {
        const int wc = (int)(p % a.w);
        const int64_t r = p / a.w;
        const int hr = (int)(r % a.h);
        const int64_t img = r / a.h;
        const int hh = hr + dh, ww = wc + dw;
        if (hh >= 0 && hh < a.h && ww >= 0 && ww < a.w)
          xv = (float)a.x[((img * a.h + hh) * a.w + ww) * (int64_t)a.ldx + c0 + c];
        dv = (float)a.dy[p * (int64_t)a.lddy + o0 + c];
      }
      xs[j][c] = xv;
      ds[j][c] = dv;
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < 64; ++j) {
      const float x0 = xs[j][2 * ty], x1 = xs[j][2 * ty + 1];
      const float d0 = ds[j][2 * tx], d1 = ds[j][2 * tx + 1];
      acc[0][0] = fmaf(x0, d0, acc[0][0]);
      acc[0][1] = fmaf(x0, d1, acc[0][1]);
      acc[1][0] = fmaf(x1, d0, acc[1][0]);
      acc[1][1] = fmaf(x1, d1, acc[1][1]);
    }
    __syncthreads();
  }
  float* dst = a.dw + ((int64_t)t * a.c_in + c0 + 2 * ty) * a.c_out + o0 + 2 * tx;
  atomicAdd(dst, acc[0][0]);
  atomicAdd(dst + 1, acc[0][1]);
  atomicAdd(dst + a.c_out, acc[1][0]);
  atomicAdd(dst + a.c_out + 1, acc[1][1]);
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

__global__ __launch_bounds__(256) void head_kernel(const bf16* feat, int32_t c, int64_t P, const float* w,
                                                   const float* b, const float* target, const float* weight,
                                                   float* mask, float* err, float* dz, float* loss,
                                                   float inv_count) {
  __shared__ float red[3][256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float l0 = 0.f, l1 = 0.f, l2 = 0.f;
  if (p < P) {
    float z0 = b[0], z1 = b[1];
    for (int k = 0; k < c; ++k) {
      const float f = (float)feat[p * c + k];
      z0 = fmaf(f, w[2 * k], z0);
      z1 = fmaf(f, w[2 * k + 1], z1);
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
    if (threadIdx.x < s) {
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
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
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
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
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

// Input features from the adjacent-pixel cross-spectra of a full-aperture field: one
// workgroup per frame.  Pass 1 sums the channels over the bin splits into the energy
// (S) and finds its maximum; pass 2 writes the eight feature channels of every pixel.
// A pair's normalised cross-spectrum is taken at its even member (left column, upper
// depth), so both pixels of a pair see the same oriented value.
__global__ __launch_bounds__(1024) void coherence_features_kernel(const float* acc, int32_t n_split, int64_t sstride,
                                                                  int32_t n_z, int32_t n_x, bf16* out, float* energy) {
  __shared__ float red[1024];
  const int64_t f = blockIdx.x;
  const int64_t P = (int64_t)n_z * n_x;
  const float* a0 = acc + f * 5 * P;
  float* e = energy + f * P;
  auto chan = [&](int c, int64_t p) {
    float v = 0.f;
    for (int s = 0; s < n_split; ++s) v += a0[s * sstride + c * P + p];
    return v;
  };
  float m = 0.f;
  for (int64_t p = threadIdx.x; p < P; p += 1024) {
    const float v = chan(0, p);
    e[p] = v;
    m = fmaxf(m, v);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float inv = red[0] > 0.f ? 1.f / red[0] : 1.f;
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
  for (int64_t p = threadIdx.x; p < P; p += 1024) {
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
    if (threadIdx.x < s) {
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
    if (threadIdx.x < s) {
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

}  // namespace

extern "C" {

pam_status_t pam_nn_conv3x3(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t k_in,
                            const void* wt, const float* bias, void* y, int32_t ldy, int32_t n_out, int32_t relu,
                            int32_t flip, int32_t accumulate, void* hip_stream) {
  if (!x || !wt || !y || batch < 1 || h < 1 || w < 32 || w % 32 || k_in < 16 || k_in % 16 || n_out < 32 ||
      n_out % 32 || ldx < k_in || ldx % 8 || ldy < n_out || !aligned16(x) || !aligned16(wt))
    return PAM_ERR_INVALID_ARG;
  ConvArgs a{static_cast<const bf16*>(x), static_cast<const bf16*>(wt), bias, static_cast<bf16*>(y),
             (int64_t)batch * h * w, ldx, h, w, k_in, ldy, n_out, relu, flip, accumulate};
  const int64_t tiles = a.P / 32;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // 32 pixels x 32 NT output channels per wave
  if (n_out % 128 == 0)
    hipLaunchKernelGGL(conv3x3_kernel<4>, dim3(blocks_for(tiles, 4), n_out / 128), dim3(256), 0, st, a);
  else if (n_out % 64 == 0)
    hipLaunchKernelGGL(conv3x3_kernel<2>, dim3(blocks_for(tiles, 4), n_out / 64), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(conv3x3_kernel<1>, dim3(blocks_for(tiles, 4), n_out / 32), dim3(256), 0, st, a);
  return launched();
}

pam_status_t pam_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy, int32_t batch, int32_t h,
                                  int32_t w, int32_t c_in, int32_t c_out, float* dw, float* db, void* hip_stream) {
  if (!x || !dy || !dw || batch < 1 || h < 1 || w < 1 || c_in < 32 || c_in % 32 || c_out < 32 || c_out % 32 ||
      ldx < c_in || lddy < c_out)
    return PAM_ERR_INVALID_ARG;
  const int64_t P = (int64_t)batch * h * w;
  const int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(64, P / 4096));
  const int64_t chunk = ((P + n_chunks - 1) / n_chunks + 63) / 64 * 64;
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
  hipLaunchKernelGGL(maxpool_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), static_cast<const bf16*>(dy), lddy, arg, n, h, w, c,
                     static_cast<bf16*>(dx), lddx, accumulate);
  return launched();
}

pam_status_t pam_nn_upsample(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t c, void* y,
                             int32_t ldy, void* hip_stream) {
  if (!x || !y || batch < 1 || h < 1 || w < 1 || c < 1 || ldx < c || ldy < c) return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * 4 * h * w * c;
  hipLaunchKernelGGL(upsample_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const bf16*>(x), ldx, n, h, w, c, static_cast<bf16*>(y), ldy);
  return launched();
}

pam_status_t pam_nn_upsample_backward(const void* dy, int32_t lddy, int32_t batch, int32_t h, int32_t w, int32_t c,
                                      void* dx, int32_t lddx, void* hip_stream) {
  if (!dy || !dx || batch < 1 || h < 1 || w < 1 || c < 1 || lddy < c || lddx < c) return PAM_ERR_INVALID_ARG;
  const int64_t n = (int64_t)batch * h * w * c;
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
                                       int32_t n_z, int32_t n_x, void* out, float* energy, void* hip_stream) {
  if (!accum || !out || !energy || n_split < 1 || batch < 1 || n_z < 2 || n_x < 2 || (n_z & 1) || (n_x & 1) ||
      (n_split > 1 && split_stride < (int64_t)batch * 5 * n_z * n_x) || !aligned16(out))
    return PAM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(coherence_features_kernel, dim3(batch), dim3(1024), 0, static_cast<hipStream_t>(hip_stream), accum,
                     n_split, split_stride, n_z, n_x, static_cast<bf16*>(out), energy);
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
