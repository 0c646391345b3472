// Exhaustive pyramid-distance candidate search (Sec. 2.4.3-2.4.4, Eq. 2.22-
// 2.24) on gfx950.
//
// For a candidate window the corner grid of the finest pyramid level,
// (2^(levels-1)+1)^2 points, is read once per plane; every cell of every
// level is a four-corner difference on that grid.
//   bin-major layout: a workgroup takes 64 consecutive candidates (one per
//     lane) and splits the planes over its wavefronts.  Candidates given in
//     row-major grid order put consecutive columns in consecutive lanes, so
//     each corner read is one contiguous run across the wavefront; partial
//     sums are combined over wavefronts in a fixed order through LDS.
//   planes-innermost layout: a wavefront takes one candidate and its lanes
//     take the planes, so each corner read is one contiguous run of planes;
//     the lanes' sums are combined by a fixed butterfly.
// Results do not depend on scheduling.  A second single-workgroup kernel
// picks the best candidate (lowest index among equals).
#include <math.h>

#include "ih_internal.h"

namespace ih {

constexpr int kMatchWaves = 4;

// Per-level accumulation of one plane's cells against the template.
template <int LEVELS, int METRIC>
__device__ __forceinline__ void score_cells(const int32_t (&v)[(1 << (LEVELS - 1)) + 1][(1 << (LEVELS - 1)) + 1],
                                            const int32_t *__restrict__ tmpl, int P, int p, double (&accf)[LEVELS],
                                            int64_t (&acci)[LEVELS]) {
  constexpr int G = 1 << (LEVELS - 1);
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
        const int y = tmpl[(int64_t)k * P + p];
        if constexpr (METRIC == IH_CHI2) {
          const int sum = x + y;
          if (sum > 0) {
            const float d = (float)(x - y);
            accf[l] += (double)(d * d / (float)sum);
          }
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

template <int LEVELS, int METRIC>
__global__ __launch_bounds__(64 * kMatchWaves) void k_match(const int32_t *__restrict__ ih, int P, int H, int W,
                                                           const int32_t *__restrict__ tmpl, int win_h,
                                                           int win_w, const int32_t *__restrict__ origins,
                                                           int64_t n, float *__restrict__ dist) {
  constexpr int G = 1 << (LEVELS - 1);
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
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
          v[a][b] = (rr < 0 || cc < 0) ? 0 : ih[po + (int64_t)rr * W + cc];
        }
      }
      score_cells<LEVELS, METRIC>(v, tmpl, P, p, accf, acci);
    }
  }

  __shared__ double partf[kMatchWaves][64];
  __shared__ long long parti[kMatchWaves][64];
  double tf;
  int64_t ti;
  weigh<LEVELS>(accf, acci, tf, ti);
  partf[wave][lane] = tf;
  parti[wave][lane] = ti;
  __syncthreads();
  if (wave == 0 && q < n) {
    float res;
    if (!ok) {
      res = METRIC == IH_PMK ? -INFINITY : INFINITY;
    } else {
      double sf = 0.0;
      long long si = 0;
      for (int w = 0; w < kMatchWaves; ++w) { sf += partf[w][lane]; si += parti[w][lane]; }
      res = finish<LEVELS, METRIC>(sf, si);
    }
    dist[q] = res;
  }
}

template <int LEVELS, int METRIC>
__global__ __launch_bounds__(256) void k_match_hwb(const int32_t *__restrict__ ih, int P, int H, int W,
                                                  const int32_t *__restrict__ tmpl, int win_h, int win_w,
                                                  const int32_t *__restrict__ origins, int64_t n,
                                                  float *__restrict__ dist) {
  constexpr int G = 1 << (LEVELS - 1);
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
  if (q >= n) return;
  const int r = origins[2 * q], c = origins[2 * q + 1];
  if (!(r >= 0 && c >= 0 && (int64_t)r + win_h <= H && (int64_t)c + win_w <= W)) {
    if (lane == 0) dist[q] = METRIC == IH_PMK ? -INFINITY : INFINITY;
    return;
  }
  int64_t off[G + 1][G + 1];  // element offsets of the corner grid; -1 reads as 0
#pragma unroll
  for (int a = 0; a <= G; ++a) {
    const int rr = r + (int)((int64_t)a * win_h / G) - 1;
#pragma unroll
    for (int b = 0; b <= G; ++b) {
      const int cc = c + (int)((int64_t)b * win_w / G) - 1;
      off[a][b] = (rr < 0 || cc < 0) ? -1 : ((int64_t)rr * W + cc) * P;
    }
  }
  double accf[LEVELS];
  int64_t acci[LEVELS];
#pragma unroll
  for (int l = 0; l < LEVELS; ++l) { accf[l] = 0.0; acci[l] = 0; }
  for (int p = lane; p < P; p += 64) {
    int32_t v[G + 1][G + 1];
#pragma unroll
    for (int a = 0; a <= G; ++a)
#pragma unroll
      for (int b = 0; b <= G; ++b) v[a][b] = off[a][b] < 0 ? 0 : ih[off[a][b] + p];
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

// Best candidate: smallest distance (largest for PMK), lowest index on ties;
// infinite scores are out-of-frame candidates and never chosen.
template <bool LARGEST>
__global__ __launch_bounds__(1024) void k_argbest(const float *__restrict__ dist, int64_t n,
                                                 int32_t *__restrict__ best) {
  __shared__ float sv[1024];
  __shared__ int64_t si[1024];
  float bv = 0.0f;
  int64_t bi = -1;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float v = dist[i];
    if (isinf(v)) continue;
    if (bi < 0 || (LARGEST ? v > bv : v < bv)) { bv = v; bi = i; }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
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

typedef void (*match_fn)(const int32_t *, int, int, int, const int32_t *, int, int, const int32_t *, int64_t,
                         float *);

template <int LEVELS>
static match_fn pick_metric(int metric, bool hwb) {
  if (hwb) {
    if (metric == IH_CHI2) return &k_match_hwb<LEVELS, IH_CHI2>;
    if (metric == IH_L1) return &k_match_hwb<LEVELS, IH_L1>;
    return &k_match_hwb<LEVELS, IH_PMK>;
  }
  if (metric == IH_CHI2) return &k_match<LEVELS, IH_CHI2>;
  if (metric == IH_L1) return &k_match<LEVELS, IH_L1>;
  return &k_match<LEVELS, IH_PMK>;
}

static match_fn pick_match(int levels, int metric, bool hwb) {
  switch (levels) {
    case 1: return pick_metric<1>(metric, hwb);
    case 2: return pick_metric<2>(metric, hwb);
    case 3: return pick_metric<3>(metric, hwb);
    default: return pick_metric<4>(metric, hwb);
  }
}

}  // namespace ih

using namespace ih;

extern "C" int ih_match_candidates(const int32_t *ihp, int32_t P, int32_t H, int32_t W, int32_t layout,
                                   const int32_t *tmpl_desc, int32_t win_h, int32_t win_w, int32_t levels,
                                   const int32_t *origins, int64_t n, int32_t metric, float *dist, int32_t *best,
                                   void *stream) {
  if (P < 1 || H < 1 || W < 1) return set_error(IH_ERR_INVALID_ARG, "P, H, W must be positive");
  if (layout != IH_BHW && layout != IH_HWB) return set_error(IH_ERR_INVALID_ARG, "layout %d unknown", layout);
  if (win_h < 1 || win_w < 1) return set_error(IH_ERR_INVALID_ARG, "window %dx%d must be positive", win_h, win_w);
  if (levels < 1 || levels > 4) return set_error(IH_ERR_INVALID_ARG, "levels %d outside 1..4", levels);
  if (metric != IH_CHI2 && metric != IH_L1 && metric != IH_PMK)
    return set_error(IH_ERR_INVALID_ARG, "metric %d unknown", metric);
  if (n < 0 || n >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "n=%lld outside 0..2^31-1", (long long)n);
  if (!ihp || !tmpl_desc || !origins || !dist || !best) return set_error(IH_ERR_INVALID_ARG, "NULL pointer");
  hipStream_t s = as_stream(stream);
  int e;
  if (n > 0) {
    const bool hwb = layout == IH_HWB;
    match_fn f = pick_match(levels, metric, hwb);
    const dim3 grid = hwb ? dim3((unsigned)((n + 3) / 4)) : dim3((unsigned)((n + 63) / 64));
    const dim3 block = hwb ? dim3(256) : dim3(64 * kMatchWaves);
    hipLaunchKernelGGL(f, grid, block, 0, s, ihp, P, H, W, tmpl_desc, win_h, win_w, origins, n, dist);
    if ((e = hip_check(hipGetLastError(), "match launch"))) return e;
  }
  if (metric == IH_PMK)
    hipLaunchKernelGGL(k_argbest<true>, dim3(1), dim3(1024), 0, s, dist, n, best);
  else
    hipLaunchKernelGGL(k_argbest<false>, dim3(1), dim3(1024), 0, s, dist, n, best);
  return hip_check(hipGetLastError(), "argbest launch");
}
