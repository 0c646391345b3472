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
#include "ih_match_dev.h"

namespace ih {

template <int LEVELS, int METRIC>
__global__ __launch_bounds__(64 * kMatchWaves) void k_match(const int32_t *__restrict__ ih, int P, int H, int W,
                                                           const int32_t *__restrict__ tmpl, int win_h,
                                                           int win_w, const int32_t *__restrict__ origins,
                                                           int64_t n, float *__restrict__ dist) {
  __shared__ double partf[kMatchWaves * 64];
  __shared__ long long parti[kMatchWaves * 64];
  match_body<LEVELS, METRIC>(ih, P, H, W, tmpl, win_h, win_w, origins, n, dist, blockIdx.x, partf, parti);
}

template <bool LARGEST>
__global__ __launch_bounds__(1024) void k_argbest(const float *__restrict__ dist, int64_t n,
                                                 int32_t *__restrict__ best) {
  __shared__ float sv[1024];
  __shared__ int64_t si[1024];
  argbest_body<LARGEST>(dist, n, best, sv, si);
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
  // planes-innermost corner offsets within a pixel row are 32-bit
  if (layout == IH_HWB && (int64_t)W * P > 0xffffffffLL)
    return set_error(IH_ERR_RANGE, "W*P=%lld above 2^32-1 planes-innermost", (long long)W * P);
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
