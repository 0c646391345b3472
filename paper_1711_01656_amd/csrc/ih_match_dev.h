// Device bodies of the pyramid-distance search, shared by the stand-alone
// kernels (ih_match.hip) and the persistent batched kernel (ih_batch.hip).
#pragma once

#include <math.h>

#include "ih_internal.h"

namespace ih {

constexpr int kMatchWaves = 4;

// All cells of the LEVELS-level pyramid descriptor of window w = {r, c, h, w}
// for plane p (Alg. 2, Sec. 2.4.4): the corner grid of the finest level is
// read once and every cell is a four-corner difference on it.  o points at
// cell 0 of plane p; cell k is written at o[k * P].  Windows not inside the
// frame give -1.
template <int LEVELS>
__device__ __forceinline__ void pyramid_cells(const int32_t *__restrict__ ih, int P, int H, int W, int layout,
                                              const int32_t *__restrict__ win, int p, int32_t *__restrict__ o) {
  constexpr int G = 1 << (LEVELS - 1);
  constexpr int CELLS = ((1 << (2 * LEVELS)) - 1) / 3;
  const int r = win[0], c = win[1], h = win[2], w = win[3];
  const bool ok = h >= 1 && w >= 1 && r >= 0 && c >= 0 && (int64_t)r + h <= H && (int64_t)c + w <= W;
  if (!ok) {
    for (int k = 0; k < CELLS; ++k) o[k * P] = -1;
    return;
  }
  const Addr A(layout, p, P, H, W);
  int32_t v[G + 1][G + 1];
#pragma unroll
  for (int a = 0; a <= G; ++a)
#pragma unroll
    for (int b = 0; b <= G; ++b)
      v[a][b] = A.at(ih, r + (int)((int64_t)a * h / G) - 1, c + (int)((int64_t)b * w / G) - 1);
  int k = 0;
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) {
    const int s = G >> l;
#pragma unroll
    for (int a = 0; a < (1 << l); ++a)
#pragma unroll
      for (int b = 0; b < (1 << l); ++b, ++k)
        o[k * P] = v[(a + 1) * s][(b + 1) * s] - v[a * s][(b + 1) * s] - v[(a + 1) * s][b * s] + v[a * s][b * s];
  }
}

// Per-level accumulation of one plane's cells against the template.
template <int LEVELS, int METRIC>
__device__ __forceinline__ void score_cells(const int32_t (&v)[(1 << (LEVELS - 1)) + 1][(1 << (LEVELS - 1)) + 1],
                                            const int32_t *__restrict__ tmpl, int P, int p, double (&accf)[LEVELS],
                                            int64_t (&acci)[LEVELS]) {
  constexpr int G = 1 << (LEVELS - 1);
  constexpr int CELLS = ((1 << (2 * LEVELS)) - 1) / 3;
  int ty[CELLS];  // the template's cells of this plane, all loads issued first
#pragma unroll
  for (int k = 0; k < CELLS; ++k) ty[k] = tmpl[(int64_t)k * P + p];
  int k = 0;
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) {
    const int s = G >> l;
    int64_t li = 0;
#pragma unroll
    for (int a = 0; a < (1 << l); ++a)
#pragma unroll
      for (int b = 0; b < (1 << l); ++b, ++k) {
        const int x = v[(a + 1) * s][(b + 1) * s] - v[a * s][(b + 1) * s] - v[(a + 1) * s][b * s] + v[a * s][b * s];
        const int y = ty[k];
        if constexpr (METRIC == IH_CHI2) {
          // branch-free, so the template loads of all cells can be issued
          // together; a cell with x + y = 0 adds +0.0, which leaves the
          // non-negative sum unchanged
          const int sum = x + y;
          const float d = (float)(x - y);
          const float t = d * d / (float)(sum > 0 ? sum : 1);
          accf[l] += sum > 0 ? (double)t : 0.0;
        } else if constexpr (METRIC == IH_L1) {
          li += x > y ? x - y : y - x;
        } else {
          li += x < y ? x : y;
        }
      }
    acci[l] += li;
  }
}

// Level weights of Eq. 2.24 (level 0: 1/2^L, level l >= 1: 1/2^(L-l+1));
// integer metrics are scaled by 2^L to stay exact (weights 1, 1, 2, 4, ...).
template <int LEVELS>
__device__ __forceinline__ void weigh(const double (&accf)[LEVELS], const int64_t (&acci)[LEVELS], double &tf,
                                      int64_t &ti) {
  tf = 0.0;
  ti = 0;
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) {
    const int L = LEVELS - 1;
    tf += (l == 0 ? ldexp(1.0, -L) : ldexp(1.0, -(L - l + 1))) * accf[l];
    ti += (l == 0 ? 1LL : (1LL << (l - 1))) * acci[l];
  }
}

template <int LEVELS, int METRIC>
__device__ __forceinline__ float finish(double tf, int64_t ti) {
  if (METRIC == IH_CHI2) return (float)tf;
  return (float)ldexp((double)ti, -(LEVELS - 1));
}

// Bin-major search: block `blk` takes candidates blk*64 .. blk*64+63; the
// block's kMatchWaves wavefronts split the planes.  partf / parti are LDS
// arrays of kMatchWaves*64 entries.
template <int LEVELS, int METRIC>
__device__ __forceinline__ void match_body(const int32_t *__restrict__ ih, int P, int H, int W,
                                           const int32_t *__restrict__ tmpl, int win_h, int win_w,
                                           const int32_t *__restrict__ origins, int64_t n, float *__restrict__ dist,
                                           int64_t blk, double *partf, long long *parti) {
  constexpr int G = 1 << (LEVELS - 1);
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int64_t q = blk * 64 + lane;
  int r = 0, c = 0;
  bool ok = false;
  if (q < n) {
    r = origins[2 * q];
    c = origins[2 * q + 1];
    ok = r >= 0 && c >= 0 && (int64_t)r + win_h <= H && (int64_t)c + win_w <= W;
  }
  int ro[G + 1], co[G + 1];
#pragma unroll
  for (int i = 0; i <= G; ++i) {
    ro[i] = (int)((int64_t)i * win_h / G);
    co[i] = (int)((int64_t)i * win_w / G);
  }
  double accf[LEVELS];
  int64_t acci[LEVELS];
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) { accf[l] = 0.0; acci[l] = 0; }

  for (int p = wave; p < P; p += kMatchWaves) {
    if (ok) {
      const int64_t po = (int64_t)p * H * W;
      int32_t v[G + 1][G + 1];
#pragma unroll
      for (int a = 0; a <= G; ++a) {
        const int rr = r + ro[a] - 1;
#pragma unroll
        for (int b = 0; b <= G; ++b) {
          const int cc = c + co[b] - 1;
          const int32_t x = ih[po + (int64_t)max(rr, 0) * W + max(cc, 0)];  // unconditional load
          v[a][b] = (rr < 0 || cc < 0) ? 0 : x;
        }
      }
      score_cells<LEVELS, METRIC>(v, tmpl, P, p, accf, acci);
    }
  }

  double tf;
  int64_t ti;
  weigh<LEVELS>(accf, acci, tf, ti);
  partf[wave * 64 + lane] = tf;
  parti[wave * 64 + lane] = ti;
  __syncthreads();
  if (wave == 0 && q < n) {
    float res;
    if (!ok) {
      res = METRIC == IH_PMK ? -INFINITY : INFINITY;
    } else {
      double sf = 0.0;
      long long si = 0;
      for (int w = 0; w < kMatchWaves; ++w) { sf += partf[w * 64 + lane]; si += parti[w * 64 + lane]; }
      res = finish<LEVELS, METRIC>(sf, si);
    }
    dist[q] = res;
  }
}

// Planes-innermost search: one wavefront per candidate q, lanes over planes.
template <int LEVELS, int METRIC>
__device__ __forceinline__ void match_hwb_body(const int32_t *__restrict__ ih, int P, int H, int W,
                                               const int32_t *__restrict__ tmpl, int win_h, int win_w,
                                               const int32_t *__restrict__ origins, int64_t n,
                                               float *__restrict__ dist, int64_t q) {
  constexpr int G = 1 << (LEVELS - 1);
  const int lane = threadIdx.x & 63;
  if (q >= n) return;
  const int r = origins[2 * q], c = origins[2 * q + 1];
  if (!(r >= 0 && c >= 0 && (int64_t)r + win_h <= H && (int64_t)c + win_w <= W)) {
    if (lane == 0) dist[q] = METRIC == IH_PMK ? -INFINITY : INFINITY;
    return;
  }
  // Corner grid as wave-uniform row pointers and 32-bit column offsets;
  // corners on the virtual row/column -1 (only grid row 0 when r = 0, grid
  // column 0 when c = 0) are read from row/column 0 and masked to zero, so
  // every load is unconditional and the loads of a plane can all be in
  // flight together.
  const int32_t *rowp[G + 1];
  uint32_t colo[G + 1];
#pragma unroll
  for (int a = 0; a <= G; ++a) {
    const int rr = r + (int)((int64_t)a * win_h / G) - 1;
    rowp[a] = ih + (int64_t)max(rr, 0) * W * P;
  }
#pragma unroll
  for (int b = 0; b <= G; ++b) {
    const int cc = c + (int)((int64_t)b * win_w / G) - 1;
    colo[b] = (uint32_t)max(cc, 0) * (uint32_t)P;
  }
  const int32_t mrow = r > 0 ? -1 : 0, mcol = c > 0 ? -1 : 0;
  double accf[LEVELS];
  int64_t acci[LEVELS];
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) { accf[l] = 0.0; acci[l] = 0; }
  for (int p = lane; p < P; p += 64) {
    int32_t v[G + 1][G + 1];
#pragma unroll
    for (int a = 0; a <= G; ++a)
#pragma unroll
      for (int b = 0; b <= G; ++b) {
        const int32_t x = rowp[a][colo[b] + (uint32_t)p];
        v[a][b] = a == 0 ? (b == 0 ? x & mrow & mcol : x & mrow) : (b == 0 ? x & mcol : x);
      }
    score_cells<LEVELS, METRIC>(v, tmpl, P, p, accf, acci);
  }
  double tf;
  int64_t ti;
  weigh<LEVELS>(accf, acci, tf, ti);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    tf += __shfl_xor(tf, m, 64);
    ti += __shfl_xor((long long)ti, m, 64);
  }
  if (lane == 0) dist[q] = finish<LEVELS, METRIC>(tf, ti);
}

template <int LEVELS, int METRIC>
__global__ __launch_bounds__(256) void k_match_hwb(const int32_t *__restrict__ ih, int P, int H, int W,
                                                  const int32_t *__restrict__ tmpl, int win_h, int win_w,
                                                  const int32_t *__restrict__ origins, int64_t n,
                                                  float *__restrict__ dist) {
  match_hwb_body<LEVELS, METRIC>(ih, P, H, W, tmpl, win_h, win_w, origins, n, dist,
                                 (int64_t)blockIdx.x * (blockDim.x >> 6) + uniform(threadIdx.x >> 6));
}

// Best candidate: smallest distance (largest for PMK), lowest index on ties;
// infinite scores are out-of-frame candidates and never chosen.
// One block: sv / si are LDS arrays of blockDim.x (a power of two) entries.
template <bool LARGEST>
__device__ __forceinline__ void argbest_body(const float *__restrict__ dist, int64_t n, int32_t *__restrict__ best,
                                             float *sv, int64_t *si) {
  float bv = 0.0f;
  int64_t bi = -1;
  // 8 loads in flight per thread (indexes clamped to n-1, the values past
  // the end ignored), then compared in increasing index order
  constexpr int U = 8;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)U * blockDim.x) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      v[u] = dist[i < n ? i : n - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      if (i < n && !isinf(v[u]) && (bi < 0 || (LARGEST ? v[u] > bv : v[u] < bv))) { bv = v[u]; bi = i; }
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const float ov = sv[threadIdx.x + s];
      const int64_t oi = si[threadIdx.x + s];
      const int64_t mi = si[threadIdx.x];
      const float mv = sv[threadIdx.x];
      bool take = false;
      if (oi >= 0) {
        if (mi < 0) take = true;
        else if (LARGEST ? ov > mv : ov < mv) take = true;
        else if (ov == mv && oi < mi) take = true;
      }
      if (take) { sv[threadIdx.x] = ov; si[threadIdx.x] = oi; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = (int32_t)si[0];
}


}  // namespace ih
