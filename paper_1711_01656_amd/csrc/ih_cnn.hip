// Learned candidate proposal: a small BF16 convolutional network trained and
// run by these kernels (gfx950).
//
//   x  (7x128x128) -conv 3x3 s2-> a1 (32x64x64) -conv 3x3 d3-> a2 -conv 3x3 d9-> a3
//   s = wh . a3 + bh (64x64);  logits(dy,dx) = bilinear(s, 32 + dy/2, 32 + dx/2)
//
// Convolutions, their input gradients and their weight gradients are implicit
// GEMMs on the 32x32x8 BF16 matrix cores with FP32 accumulation:
//   forward  out[co][pix] = sum_k W[co][k] X[k][pix]      (M=32, N=pixels, K=9*Cpad)
//   dgrad    the forward of dZ with W transposed and its taps flipped
//   wgrad    dW[co][k]     = sum_pix dZ[co][pix] X[k][pix] (M=32, N=K, K=pixels)
// X is the im2col view of the layer input, gathered on the fly.  Reductions
// over pixels run in a fixed order, so results do not depend on scheduling.
#include "ih_internal.h"
#include "ih_lp.h"

namespace ih {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int LP_CO = 32;    // output channels of every convolution
constexpr int LP_SMAP = 64;  // score map side
constexpr int LP_R = 32;     // offsets per side: -32 .. 32
constexpr int LP_NOFF = 2 * LP_R + 1;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct ConvShape {
  int B, Cin, Hin, Win, Hout, Wout, stride, dil, pad;
  int K, Kpad;   // weight gradients: K = Cin*9 (channel-major), Kpad = K rounded up to 8
  int Cpad, Kt;  // convolutions: channels padded to 8, Kt = 9*Cpad (tap-major)
};

// Value of the im2col matrix X[k][pixel] for the pixel (b, y, x), extended by
// a column of ones at k = K (its product with dZ is the bias gradient).
__device__ __forceinline__ short im2col(const uint16_t *__restrict__ in, const ConvShape &s, int k, int b, int y,
                                        int x) {
  if (k >= s.K) return k == s.K ? (short)0x3f80 : (short)0;  // bf16 1.0
  const int ci = k / 9, t = k - ci * 9, kh = t / 3, kw = t - kh * 3;
  const int r = y * s.stride + kh * s.dil - s.pad, c = x * s.stride + kw * s.dil - s.pad;
  if (r < 0 || c < 0 || r >= s.Hin || c >= s.Win) return 0;
  return (short)in[(((int64_t)b * s.Cin + ci) * s.Hin + r) * s.Win + c];
}

// Forward convolution (also used for input gradients).  A block owns one
// tile of 32 consecutive output pixels x 32 output channels; its 4 waves split
// the K = 9*Cpad reduction (taps outer, 8 channels of one tap per matrix
// instruction, so each lane computes its source pixel once per instruction
// and needs no division), and the four partial tiles are added in a fixed
// order through LDS.
//   mask == nullptr: out = bf16(relu(acc + bias))
//   mask != nullptr: out = bf16(acc * (mask > 0))   (input gradient through a ReLU)
__global__ __launch_bounds__(256) void k_lp_conv(const uint16_t *__restrict__ in, const uint16_t *__restrict__ w,
                                                 const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                                 uint16_t *__restrict__ out, ConvShape s) {
  __shared__ float red[4][LP_CO * 32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  const int64_t npix = (int64_t)s.B * s.Hout * s.Wout;
  const int64_t p = (int64_t)blockIdx.x * 32 + (lane & 31);
  const bool live = p < npix;
  const int64_t pc = live ? p : 0;
  const int x = (int)(pc % s.Wout), y = (int)((pc / s.Wout) % s.Hout), b = (int)(pc / ((int64_t)s.Wout * s.Hout));
  const int64_t plane = (int64_t)s.Hin * s.Win;
  const uint16_t *inb = in + (int64_t)b * s.Cin * plane;
  const uint16_t *wrow = w + (int64_t)(lane & 31) * s.Kt + 4 * half;
  const int groups = s.Cpad >> 3, nslice = s.Kt >> 3;
  const int per = (nslice + 3) >> 2;
  const int s0 = wave * per, s1 = min(nslice, s0 + per);
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int sl = s0; sl < s1; ++sl) {
    const int t = sl / groups, ci0 = (sl - t * groups) * 8 + 4 * half;
    const int kh = t / 3, kw = t - kh * 3;
    const int r = y * s.stride + kh * s.dil - s.pad, c = x * s.stride + kw * s.dil - s.pad;
    const bool inside = live && r >= 0 && c >= 0 && r < s.Hin && c < s.Win;
    const bf16x4 a = *reinterpret_cast<const bf16x4 *>(wrow + sl * 8);
    bf16x4 bv;
    const int64_t off = (int64_t)ci0 * plane + (int64_t)r * s.Win + c;
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = inside && ci0 + j < s.Cin ? (short)inb[off + j * plane] : (short)0;
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][(8 * (r >> 2) + 4 * half + (r & 3)) * 32 + (lane & 31)] = acc[r];
  __syncthreads();
  for (int e = threadIdx.x; e < LP_CO * 32; e += 256) {
    const int co = e >> 5;
    const int64_t q = (int64_t)blockIdx.x * 32 + (e & 31);
    if (q >= npix) continue;
    float v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    const int xq = (int)(q % s.Wout), yq = (int)((q / s.Wout) % s.Hout), bq = (int)(q / ((int64_t)s.Wout * s.Hout));
    const int64_t o = (((int64_t)bq * LP_CO + co) * s.Hout + yq) * s.Wout + xq;
    if (mask) {
      v = bf2f(mask[o]) > 0.0f ? v : 0.0f;
    } else {
      v += bias[co];
      v = v > 0.0f ? v : 0.0f;
    }
    out[o] = f2bf(v);
  }
}

// Weight-gradient partial sums.  Block (kt, chunk) owns a 32 (co) x 32 (k)
// tile of dW = sum_pixels dZ[co][pixel] X[k][pixel] over one chunk of output
// pixels, k = kt .. kt+31 (k = K is the column of ones: the bias gradient).
// The chunk is walked in steps of kWgStep pixels: each thread decodes its
// pixel once per step and stages that pixel's dZ column (32 channels) and
// im2col column (the tile's 32 k) in LDS, loads coalesced along the row;
// then each wave runs the matrix instructions over its quarter of the step
// (8 pixels per instruction), its accumulator carried across steps.  The four
// waves' tiles are added in a fixed order and written to part[chunk][co][k].
constexpr int kWgStep = 256;
constexpr int kWgLd = kWgStep + 4;  // LDS row of one channel / k: 8 bytes of padding keep b64 reads conflict-free

__global__ __launch_bounds__(256) void k_lp_wgrad(const uint16_t *__restrict__ in, const uint16_t *__restrict__ dz,
                                                  float *__restrict__ part, ConvShape s, int64_t chunk) {
  constexpr int kStageBytes = 2 * 32 * kWgLd * 2;
  constexpr int kRedBytes = 4 * LP_CO * 32 * 4;
  __shared__ __align__(16) unsigned char lds[kStageBytes > kRedBytes ? kStageBytes : kRedBytes];
  uint16_t *zs = reinterpret_cast<uint16_t *>(lds);
  uint16_t *xs = zs + 32 * kWgLd;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5;
  const int kt = blockIdx.x * 32;
  const int64_t hw = (int64_t)s.Hout * s.Wout;
  const int64_t npix = (int64_t)s.B * hw;
  const int64_t p_begin = (int64_t)blockIdx.y * chunk;
  const int64_t p_end = p_begin + chunk < npix ? p_begin + chunk : npix;
  const int64_t in_plane = (int64_t)s.Hin * s.Win;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int64_t p0 = p_begin; p0 < p_end; p0 += kWgStep) {
    const int64_t p = p0 + tid;
    const bool live = p < p_end;
    int b = 0, y = 0, x = 0;
    if (live) {
      const int64_t q = p / s.Wout;
      x = (int)(p - q * s.Wout);
      b = (int)(q / s.Hout);
      y = (int)(q - (int64_t)b * s.Hout);
    }
    __syncthreads();  // the previous step's operands have been read
    {
      const uint16_t *zp = dz + ((int64_t)b * LP_CO * s.Hout + y) * s.Wout + x;
#pragma unroll 8
      for (int co = 0; co < LP_CO; ++co) zs[co * kWgLd + tid] = live ? zp[co * hw] : (uint16_t)0;
    }
    {
      const uint16_t *ib = in + (int64_t)b * s.Cin * in_plane;
      const int ry = y * s.stride - s.pad, rx = x * s.stride - s.pad;
#pragma unroll 4
      for (int kk = 0; kk < 32; ++kk) {
        const int k = kt + kk;  // wave-uniform
        uint16_t v = 0;
        if (k < s.K) {
          const int ci = k / 9, t = k - ci * 9, kh = t / 3, kw = t - kh * 3;
          const int r = ry + kh * s.dil, c = rx + kw * s.dil;
          if (live && r >= 0 && c >= 0 && r < s.Hin && c < s.Win) v = ib[(int64_t)ci * in_plane + (int64_t)r * s.Win + c];
        } else if (k == s.K) {
          v = live ? (uint16_t)0x3f80 : (uint16_t)0;  // bf16 1.0
        }
        xs[kk * kWgLd + tid] = v;
      }
    }
    __syncthreads();
    const int cl = lane & 31;
#pragma unroll
    for (int st = 0; st < kWgStep / 4 / 8; ++st) {
      const int px = wave * (kWgStep / 4) + st * 8 + 4 * half;
      const bf16x4 av = *reinterpret_cast<const bf16x4 *>(zs + cl * kWgLd + px);
      const bf16x4 bv = *reinterpret_cast<const bf16x4 *>(xs + cl * kWgLd + px);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
  }
  __syncthreads();  // the staging area becomes the reduction area
  float(*red)[LP_CO * 32] = reinterpret_cast<float(*)[LP_CO * 32]>(lds);
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][(8 * (r >> 2) + 4 * half + (r & 3)) * 32 + (lane & 31)] = acc[r];
  __syncthreads();
  for (int i = threadIdx.x; i < LP_CO * 32; i += blockDim.x) {
    const int co = i / 32, kk = i - co * 32;
    if (kt + kk <= s.K) {
      const float v = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
      part[((int64_t)blockIdx.y * LP_CO + co) * (s.K + 1) + kt + kk] = v;
    }
  }
}

// Sum of the partial rows in row order: dw[co][k] (k < K) and db[co] (k = K).
__global__ void k_lp_sum_rows(const float *__restrict__ part, int64_t rows, int K, float *__restrict__ dw,
                              float *__restrict__ db) {
  const int64_t cols = (int64_t)LP_CO * (K + 1);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int64_t r = 0; r < rows; ++r) s += part[r * cols + j];
  const int co = (int)(j / (K + 1)), k = (int)(j - (int64_t)co * (K + 1));
  if (k < K) dw[co * K + k] = s;
  else db[co] = s;
}

// Block reduction in a fixed tree order; returns the sum in thread 0.
__device__ __forceinline__ float block_sum(float v, float *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

// Score-map value s(u, v) = wh . a3[:, u, v] + bh.
__device__ __forceinline__ float score_at(const uint16_t *__restrict__ a3, const float *__restrict__ wh, float bh,
                                          int b, int u, int v) {
  // the channel values are loaded together, then summed in channel order
  uint16_t x[LP_CO];
  const uint16_t *p = a3 + (((int64_t)b * LP_CO) * LP_SMAP + u) * LP_SMAP + v;
#pragma unroll
  for (int c = 0; c < LP_CO; ++c) x[c] = p[(int64_t)c * LP_SMAP * LP_SMAP];
  float acc = bh;
#pragma unroll
  for (int c = 0; c < LP_CO; ++c) acc += wh[c] * bf2f(x[c]);
  return acc;
}

// logits[b][dy][dx] = bilinear(s, 32 + dy/2, 32 + dx/2).
__global__ __launch_bounds__(256) void k_lp_head(const uint16_t *__restrict__ a3, const float *__restrict__ wh,
                                                 const float *__restrict__ bh, int B, float *__restrict__ logits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * LP_NOFF * LP_NOFF) return;
  const int b = (int)(i / (LP_NOFF * LP_NOFF));
  const int t = (int)(i - (int64_t)b * LP_NOFF * LP_NOFF);
  const int iy = t / LP_NOFF, ix = t - iy * LP_NOFF;  // offset + 32
  const int u0 = LP_SMAP / 2 + ((iy - LP_R) >> 1), v0 = LP_SMAP / 2 + ((ix - LP_R) >> 1);  // floor
  const bool fu = (iy - LP_R) & 1, fv = (ix - LP_R) & 1;
  const float b0 = bh[0];
  float r = score_at(a3, wh, b0, b, u0, v0);
  if (fu && fv) {
    r = 0.25f * (r + score_at(a3, wh, b0, b, u0 + 1, v0) + score_at(a3, wh, b0, b, u0, v0 + 1) +
                 score_at(a3, wh, b0, b, u0 + 1, v0 + 1));
  } else if (fu) {
    r = 0.5f * (r + score_at(a3, wh, b0, b, u0 + 1, v0));
  } else if (fv) {
    r = 0.5f * (r + score_at(a3, wh, b0, b, u0, v0 + 1));
  }
  logits[i] = r;
}

// Softmax cross-entropy per sample: loss[b] and dlogits = (softmax - onehot)/B.
__global__ __launch_bounds__(256) void k_lp_softmax_ce(const float *__restrict__ logits,
                                                       const int32_t *__restrict__ labels, int B,
                                                       float *__restrict__ loss, float *__restrict__ dlogits) {
  __shared__ float sh[256];
  const int b = blockIdx.x;
  const int n = LP_NOFF * LP_NOFF;
  const float *l = logits + (int64_t)b * n;
  float m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, l[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  m = sh[0];
  __syncthreads();
  float e = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) e += expf(l[i] - m);
  const float z = block_sum(e, sh);
  const int lab = labels[b];  // a label outside [0, n) gives a NaN loss and no one-hot term
  const bool ok = lab >= 0 && lab < n;
  if (threadIdx.x == 0) loss[b] = ok ? logf(z) + m - l[lab] : __builtin_nanf("");
  for (int i = threadIdx.x; i < n; i += 256)
    dlogits[(int64_t)b * n + i] = (expf(l[i] - m) / z - (i == lab ? 1.0f : 0.0f)) / (float)B;
}

// Head backward.  dS is gathered from the logits that sample each score cell
// (weights 1 and 1/2 on the half-pixel grid); then dZ3 = bf16(dS wh (a3 > 0)).
__global__ __launch_bounds__(256) void k_lp_head_bwd(const float *__restrict__ dlogits, const uint16_t *__restrict__ a3,
                                                     const float *__restrict__ wh, int B, float *__restrict__ ds,
                                                     uint16_t *__restrict__ dz3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * LP_SMAP * LP_SMAP) return;
  const int b = (int)(i / (LP_SMAP * LP_SMAP));
  const int t = (int)(i - (int64_t)b * LP_SMAP * LP_SMAP);
  const int u = t / LP_SMAP, v = t - u * LP_SMAP;
  const float *dl = dlogits + (int64_t)b * LP_NOFF * LP_NOFF;
  float acc = 0.0f;
  // offsets whose sampling row touches u: dy = 2(u-32) (weight 1), 2(u-32)+-1 (weight 1/2)
  for (int ey = -1; ey <= 1; ++ey) {
    const int dy = 2 * (u - LP_SMAP / 2) + ey;
    if (dy < -LP_R || dy > LP_R) continue;
    const float wy = ey == 0 ? 1.0f : 0.5f;
    for (int ex = -1; ex <= 1; ++ex) {
      const int dx = 2 * (v - LP_SMAP / 2) + ex;
      if (dx < -LP_R || dx > LP_R) continue;
      const float wx = ex == 0 ? 1.0f : 0.5f;
      acc += wy * wx * dl[(dy + LP_R) * LP_NOFF + dx + LP_R];
    }
  }
  ds[i] = acc;
  for (int c = 0; c < LP_CO; ++c) {
    const int64_t o = (((int64_t)b * LP_CO + c) * LP_SMAP + u) * LP_SMAP + v;
    dz3[o] = f2bf(bf2f(a3[o]) > 0.0f ? acc * wh[c] : 0.0f);
  }
}

// Head parameter gradients, stage 1: block b sums dS * a3[c] (c < 32) and dS
// (c = 32) over the pixels of sample b; each thread keeps 33 running sums over
// its pixels, and the 256 threads' sums are added in thread order.
__global__ __launch_bounds__(256) void k_lp_head_wgrad(const float *__restrict__ ds, const uint16_t *__restrict__ a3,
                                                       float *__restrict__ part) {
  __shared__ float red[LP_CO + 1][256];
  const int b = blockIdx.x;
  const int HW = LP_SMAP * LP_SMAP;
  float acc[LP_CO + 1];
#pragma unroll
  for (int c = 0; c <= LP_CO; ++c) acc[c] = 0.0f;
  for (int i = threadIdx.x; i < HW; i += 256) {
    const float d = ds[(int64_t)b * HW + i];
#pragma unroll
    for (int c = 0; c < LP_CO; ++c) acc[c] += d * bf2f(a3[((int64_t)b * LP_CO + c) * HW + i]);
    acc[LP_CO] += d;
  }
#pragma unroll
  for (int c = 0; c <= LP_CO; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  if (threadIdx.x <= LP_CO) {
    float v = 0.0f;
    for (int t = 0; t < 256; ++t) v += red[threadIdx.x][t];
    part[(int64_t)b * (LP_CO + 1) + threadIdx.x] = v;
  }
}

// Stage 2: sum over the samples in order.
__global__ void k_lp_head_wgrad_sum(const float *__restrict__ part, int B, float *__restrict__ dwh,
                                    float *__restrict__ dbh) {
  const int c = threadIdx.x;
  if (c > LP_CO) return;
  float v = 0.0f;
  for (int b = 0; b < B; ++b) v += part[(int64_t)b * (LP_CO + 1) + c];
  if (c < LP_CO) dwh[c] = v;
  else dbh[0] = v;
}

// Crops: x[b][c][i][j] = bf16(feat[f_b][c][cy - side/2 + i][cx - side/2 + j] / 255),
// 0 outside the frame (and for a frame index outside [0, F)).
__global__ __launch_bounds__(256) void k_lp_crop(const uint8_t *__restrict__ feat, int F, int C, int H, int W,
                                                 const int32_t *__restrict__ frames,
                                                 const int32_t *__restrict__ centers, int B, int side,
                                                 uint16_t *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)C * side * side;
  if (i >= (int64_t)B * per) return;
  const int b = (int)(i / per);
  const int64_t t = i - (int64_t)b * per;
  const int c = (int)(t / ((int64_t)side * side)), yx = (int)(t % ((int64_t)side * side));
  const int f = frames ? frames[b] : 0;
  const int r = centers[2 * b] - side / 2 + yx / side, q = centers[2 * b + 1] - side / 2 + yx % side;
  float v = 0.0f;
  if (f >= 0 && f < F && r >= 0 && q >= 0 && r < H && q < W)
    v = (float)feat[(((int64_t)f * C + c) * H + r) * W + q] / 255.0f;
  x[i] = f2bf(v);
}

// Candidate origins: origins[b][j] = base[b] + (dy, dx) of offset index o, with
// o = idx[b][j] (or o = j when idx is NULL); (dy, dx) = (o / n - r, o % n - r),
// n = 2r + 1.  An index outside [0, n^2) yields an origin far outside any frame.
__global__ void k_lp_origins(const int32_t *__restrict__ idx, int B, int k, const int32_t *__restrict__ base,
                             int radius, int32_t *__restrict__ origins) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * k) return;
  const int b = (int)(i / k), j = (int)(i - (int64_t)b * k);
  const int n = 2 * radius + 1;
  const int o = idx ? idx[i] : j;
  int r = -(1 << 30), c = -(1 << 30);
  if (o >= 0 && o < n * n) {
    r = base[2 * b] + o / n - radius;
    c = base[2 * b + 1] + o % n - radius;
  }
  origins[2 * i] = r;
  origins[2 * i + 1] = c;
}

// Parameter packing.  params (FP32): W1[32][7][3][3] b1[32] W2[32][32][3][3]
// b2[32] W3 b3 wh[32] bh[1].  Writes the BF16 operands of the convolutions in
// tap-major order, column k = (kh*3 + kw)*Cpad + ci: W1 as [32][72] (Cpad = 8,
// channel 7 zero), W2, W3 as [32][288], and for the input gradients the
// transposed, tap-flipped W2t, W3t: Wt[ci][(kh*3 + kw)*32 + co] = W[co][ci][2-kh][2-kw].
__global__ void k_lp_pack(const float *__restrict__ params, uint16_t *__restrict__ w1, uint16_t *__restrict__ w2,
                          uint16_t *__restrict__ w3, uint16_t *__restrict__ w2t, uint16_t *__restrict__ w3t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = 32 * 63, n2 = 32 * 288;
  const float *W1 = params, *W2 = params + n1 + 32, *W3 = W2 + n2 + 32;
  if (i < 32 * 72) {
    const int co = i / 72, k = i - co * 72, t = k >> 3, ci = k & 7;
    w1[i] = ci < 7 ? f2bf(W1[(co * 7 + ci) * 9 + t]) : (uint16_t)0;
  }
  if (i < n2) {
    const int row = i / 288, k = i - row * 288, t = k >> 5, col = k & 31;
    w2[i] = f2bf(W2[(row * 32 + col) * 9 + t]);  // row = co, col = ci
    w3[i] = f2bf(W3[(row * 32 + col) * 9 + t]);
    const int src = (col * 32 + row) * 9 + (8 - t);   // row = ci, col = co; tap flipped
    w2t[i] = f2bf(W2[src]);
    w3t[i] = f2bf(W3[src]);
  }
}

// v <- momentum v + (g + wd p);  p <- p - lr v.
__global__ void k_lp_sgd(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ v, int n, float lr,
                         float momentum, float wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float vi = momentum * v[i] + (g[i] + wd * p[i]);
  v[i] = vi;
  p[i] = p[i] - lr * vi;
}

// Exclusive prefix sum over the block in thread order (one value per thread);
// *total receives the block sum.  sh holds one slot per wave.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int w2 = 0; w2 < nw; ++w2) {
    const uint32_t x = sh[w2];
    before += w2 < wave ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// Monotone map of a logit to an unsigned key: a larger float gives a larger
// key, -0 and +0 are equal, NaN is below everything.
__device__ __forceinline__ uint32_t order_key(float f) {
  if (f != f) return 0u;
  uint32_t u = __float_as_uint(f);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int TK_THREADS = 1024, TK_PER = 8;  // n <= 8192

// Top-k offsets per sample (best first, ties to the lower index, NaN last).
// Radix select on the order keys: four 8-bit passes, each a histogram of the
// next digit among the keys that share the digits chosen so far, find the key
// T of the k-th best; the keys above T and the first (lowest-index) keys equal
// to T are compacted in index order, and only those k are sorted.
__global__ __launch_bounds__(1024) void k_lp_topk(const float *__restrict__ logits, int n, int k,
                                                  int32_t *__restrict__ idx) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sh[TK_THREADS / 64];
  __shared__ uint32_t s_prefix, s_need;
  __shared__ uint32_t skey[TK_THREADS];
  __shared__ int32_t sidx[TK_THREADS];
  const int t = threadIdx.x;
  const float *l = logits + (int64_t)blockIdx.x * n;
  uint32_t key[TK_PER];
  const int e0 = t * TK_PER;
#pragma unroll
  for (int j = 0; j < TK_PER; ++j) key[j] = e0 + j < n ? order_key(l[e0 + j]) : 0u;
  const int nv = min(TK_PER, max(0, n - e0));  // valid elements of this thread
  uint32_t prefix = 0, mask = 0, need = (uint32_t)k;
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (t < 256) hist[t] = 0;
    __syncthreads();
    // one atomic per run of equal digits
    int run_bin = -1;
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < TK_PER; ++j) {
      if (j < nv && (key[j] & mask) == prefix) {
        const int bin = (int)((key[j] >> shift) & 255u);
        if (bin != run_bin) {
          if (run) atomicAdd(&hist[run_bin], run);
          run_bin = bin;
          run = 0;
        }
        ++run;
      }
    }
    if (run) atomicAdd(&hist[run_bin], run);
    __syncthreads();
    if (t < 64) {
      uint32_t c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) c[q] = hist[4 * t + q];
      const uint32_t lsum = c[0] + c[1] + c[2] + c[3];
      const uint32_t incl = wave_incl_scan(lsum);
      const uint32_t total = read_lane(incl, 63);
      uint32_t above = total - incl;  // keys in bins above this lane's four
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        if (above < need && need <= above + c[q]) {
          s_prefix = prefix | ((uint32_t)(4 * t + q) << shift);
          s_need = need - above;
        }
        above += c[q];
      }
    }
    __syncthreads();
    prefix = s_prefix;
    need = s_need;
    mask |= 255u << shift;
  }
  // keys > prefix: exactly k - need of them; then `need` keys == prefix, lowest indices first
  uint32_t ngt = 0, neq = 0;
#pragma unroll
  for (int j = 0; j < TK_PER; ++j)
    if (j < nv) {
      ngt += key[j] > prefix ? 1u : 0u;
      neq += key[j] == prefix ? 1u : 0u;
    }
  uint32_t tot;
  uint32_t gt_off = block_excl_scan(ngt, sh, &tot);
  uint32_t eq_off = block_excl_scan(neq, sh, &tot);
  const uint32_t cgt = (uint32_t)k - need;
#pragma unroll
  for (int j = 0; j < TK_PER; ++j) {
    if (j >= nv) continue;
    if (key[j] > prefix) {
      skey[gt_off] = key[j];
      sidx[gt_off] = e0 + j;
      ++gt_off;
    } else if (key[j] == prefix) {
      if (eq_off < need) {
        skey[cgt + eq_off] = key[j];
        sidx[cgt + eq_off] = e0 + j;
      }
      ++eq_off;
    }
  }
  int S = 1;
  while (S < k) S <<= 1;
  if (t >= k && t < S) {
    skey[t] = 0u;
    sidx[t] = 0x7fffffff;
  }
  __syncthreads();
  // bitonic sort of the S <= 1024 selected pairs: larger key first, then lower index
  for (int size = 2; size <= S; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int j = t ^ stride;
      if (t < S && j > t) {
        const bool up = (t & size) == 0;
        const uint32_t a = skey[t], c = skey[j];
        const int32_t ia = sidx[t], ic = sidx[j];
        const bool j_better = c > a || (c == a && ic < ia);
        if (j_better == up) {
          skey[t] = c;
          skey[j] = a;
          sidx[t] = ic;
          sidx[j] = ia;
        }
      }
      __syncthreads();
    }
  }
  if (t < k) idx[(int64_t)blockIdx.x * k + t] = sidx[t];
}

static int conv_shape(int B, int Cin, int Hin, int Win, int stride, int dil, int pad, ConvShape *s) {
  if (B < 1 || Cin < 1 || Hin < 1 || Win < 1 || stride < 1 || dil < 1 || pad < 0)
    return set_error(IH_ERR_INVALID_ARG, "bad convolution shape");
  s->B = B; s->Cin = Cin; s->Hin = Hin; s->Win = Win;
  s->stride = stride; s->dil = dil; s->pad = pad;
  s->Hout = (Hin + 2 * pad - 2 * dil - 1) / stride + 1;
  s->Wout = (Win + 2 * pad - 2 * dil - 1) / stride + 1;
  if (s->Hout < 1 || s->Wout < 1) return set_error(IH_ERR_INVALID_ARG, "convolution output is empty");
  if (Cin > 512) return set_error(IH_ERR_UNSUPPORTED, "Cin > 512");
  s->K = Cin * 9;
  s->Kpad = (s->K + 7) & ~7;
  s->Cpad = (Cin + 7) & ~7;
  s->Kt = 9 * s->Cpad;
  return IH_OK;
}

}  // namespace ih

using namespace ih;

extern "C" int ih_lp_conv(const uint16_t *in, int32_t B, int32_t Cin, int32_t Hin, int32_t Win, const uint16_t *w,
                          const float *bias, int32_t stride, int32_t dil, int32_t pad, const uint16_t *mask,
                          uint16_t *out, void *stream) {
  ConvShape s;
  int e = conv_shape(B, Cin, Hin, Win, stride, dil, pad, &s);
  if (e) return e;
  if (!in || !w || !out || (!mask && !bias)) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  if ((uintptr_t)w & 7) return set_error(IH_ERR_INVALID_ARG, "weights must be 8-byte aligned");
  const int64_t npix = (int64_t)B * s.Hout * s.Wout;
  const int64_t blocks = (npix + 31) / 32;
  if (blocks >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "too many output pixels");
  hipLaunchKernelGGL(k_lp_conv, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), in, w, bias, mask, out, s);
  return hip_check(hipGetLastError(), "lp conv launch");
}

extern "C" size_t ih_lp_wgrad_workspace(int32_t B, int32_t Cin, int32_t Hin, int32_t Win, int32_t stride,
                                        int32_t dil, int32_t pad, int64_t chunk) {
  ConvShape s;
  if (conv_shape(B, Cin, Hin, Win, stride, dil, pad, &s) || chunk < 8) return 0;
  const int64_t npix = (int64_t)B * s.Hout * s.Wout;
  const int64_t nchunk = (npix + chunk - 1) / chunk;
  return (size_t)nchunk * LP_CO * (s.K + 1) * 4;
}

extern "C" int ih_lp_wgrad(const uint16_t *in, const uint16_t *dz, int32_t B, int32_t Cin, int32_t Hin, int32_t Win,
                           int32_t stride, int32_t dil, int32_t pad, int64_t chunk, float *ws, size_t ws_bytes,
                           float *dw, float *db, void *stream) {
  ConvShape s;
  int e = conv_shape(B, Cin, Hin, Win, stride, dil, pad, &s);
  if (e) return e;
  if (!in || !dz || !dw || !db || !ws) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  if (chunk < 8 || chunk % 8) return set_error(IH_ERR_INVALID_ARG, "chunk must be a positive multiple of 8");
  if (ws_bytes < ih_lp_wgrad_workspace(B, Cin, Hin, Win, stride, dil, pad, chunk))
    return set_error(IH_ERR_WORKSPACE, "wgrad workspace too small");
  const int64_t npix = (int64_t)B * s.Hout * s.Wout;
  const int64_t nchunk = (npix + chunk - 1) / chunk;
  hipStream_t st = as_stream(stream);
  if (nchunk >= 65536) return set_error(IH_ERR_RANGE, "too many pixel chunks; use a larger chunk");
  hipLaunchKernelGGL(k_lp_wgrad, dim3((unsigned)((s.K + 1 + 31) / 32), (unsigned)nchunk), dim3(256), 0, st, in, dz,
                     ws, s, chunk);
  if ((e = hip_check(hipGetLastError(), "lp wgrad launch"))) return e;
  const int64_t cols = (int64_t)LP_CO * (s.K + 1);
  hipLaunchKernelGGL(k_lp_sum_rows, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, ws, nchunk, s.K, dw, db);
  return hip_check(hipGetLastError(), "lp row-sum launch");
}

extern "C" int ih_lp_head(const uint16_t *a3, const float *wh, const float *bh, int32_t B, float *logits,
                          void *stream) {
  if (B < 1 || !a3 || !wh || !bh || !logits) return set_error(IH_ERR_INVALID_ARG, "bad head arguments");
  const int64_t n = (int64_t)B * LP_NOFF * LP_NOFF;
  hipLaunchKernelGGL(k_lp_head, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), a3, wh, bh, B,
                     logits);
  return hip_check(hipGetLastError(), "lp head launch");
}

extern "C" int ih_lp_softmax_ce(const float *logits, const int32_t *labels, int32_t B, float *loss, float *dlogits,
                                void *stream) {
  if (B < 1 || !logits || !labels || !loss || !dlogits) return set_error(IH_ERR_INVALID_ARG, "bad loss arguments");
  hipLaunchKernelGGL(k_lp_softmax_ce, dim3(B), dim3(256), 0, as_stream(stream), logits, labels, B, loss, dlogits);
  return hip_check(hipGetLastError(), "lp loss launch");
}

extern "C" int ih_lp_head_bwd(const float *dlogits, const uint16_t *a3, const float *wh, int32_t B, float *ds,
                              uint16_t *dz3, float *dwh, float *dbh, float *ws, void *stream) {
  if (B < 1 || !dlogits || !a3 || !wh || !ds || !dz3 || !dwh || !dbh || !ws)
    return set_error(IH_ERR_INVALID_ARG, "bad head-backward arguments");
  hipStream_t st = as_stream(stream);
  const int64_t n = (int64_t)B * LP_SMAP * LP_SMAP;
  hipLaunchKernelGGL(k_lp_head_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dlogits, a3, wh, B, ds, dz3);
  int e = hip_check(hipGetLastError(), "lp head-backward launch");
  if (e) return e;
  hipLaunchKernelGGL(k_lp_head_wgrad, dim3(B), dim3(256), 0, st, ds, a3, ws);
  if ((e = hip_check(hipGetLastError(), "lp head-wgrad launch"))) return e;
  hipLaunchKernelGGL(k_lp_head_wgrad_sum, dim3(1), dim3(64), 0, st, ws, B, dwh, dbh);
  return hip_check(hipGetLastError(), "lp head-wgrad sum launch");
}

extern "C" int ih_lp_crop(const uint8_t *feat, int32_t F, int32_t C, int32_t H, int32_t W,
                          const int32_t *frames, const int32_t *centers, int32_t B, int32_t side, uint16_t *x,
                          void *stream) {
  if (B < 1 || F < 1 || C < 1 || H < 1 || W < 1 || side < 2 || (side & 1) || !feat || !centers || !x)
    return set_error(IH_ERR_INVALID_ARG, "bad crop arguments");
  const int64_t n = (int64_t)B * C * side * side;
  hipLaunchKernelGGL(k_lp_crop, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), feat, F, C, H,
                     W, frames, centers, B, side, x);
  return hip_check(hipGetLastError(), "lp crop launch");
}

extern "C" int ih_lp_origins(const int32_t *idx, int32_t B, int32_t k, const int32_t *base, int32_t radius,
                             int32_t *origins, void *stream) {
  if (B < 1 || k < 1 || radius < 0 || radius > 4096 || !base || !origins)
    return set_error(IH_ERR_INVALID_ARG, "bad origin arguments");
  if (!idx && k != (2 * radius + 1) * (2 * radius + 1))
    return set_error(IH_ERR_INVALID_ARG, "without idx, k must be (2 radius + 1)^2");
  const int64_t n = (int64_t)B * k;
  hipLaunchKernelGGL(k_lp_origins, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), idx, B, k,
                     base, radius, origins);
  return hip_check(hipGetLastError(), "lp origins launch");
}

extern "C" int ih_lp_pack(const float *params, uint16_t *w1, uint16_t *w2, uint16_t *w3, uint16_t *w2t,
                          uint16_t *w3t, void *stream) {
  if (!params || !w1 || !w2 || !w3 || !w2t || !w3t) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  hipLaunchKernelGGL(k_lp_pack, dim3((32 * 288 + 255) / 256), dim3(256), 0, as_stream(stream), params, w1, w2, w3,
                     w2t, w3t);
  return hip_check(hipGetLastError(), "lp pack launch");
}

extern "C" int ih_lp_sgd(float *params, const float *grads, float *mom, int32_t n, float lr, float momentum,
                         float weight_decay, void *stream) {
  if (n < 1 || !params || !grads || !mom) return set_error(IH_ERR_INVALID_ARG, "bad SGD arguments");
  hipLaunchKernelGGL(k_lp_sgd, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), params, grads, mom, n, lr,
                     momentum, weight_decay);
  return hip_check(hipGetLastError(), "lp SGD launch");
}

extern "C" int ih_lp_topk(const float *logits, int32_t B, int32_t n, int32_t k, int32_t *idx, void *stream) {
  if (B < 1 || n < 1 || n > TK_THREADS * TK_PER || k < 1 || k > n || k > TK_THREADS || !logits || !idx)
    return set_error(IH_ERR_INVALID_ARG, "bad top-k arguments (n <= 8192, 1 <= k <= min(n, 1024))");
  hipLaunchKernelGGL(k_lp_topk, dim3(B), dim3(1024), 0, as_stream(stream), logits, n, k, idx);
  return hip_check(hipGetLastError(), "lp top-k launch");
}
