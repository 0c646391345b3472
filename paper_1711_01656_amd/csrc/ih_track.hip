// Device-resident tracking step: the state of one target (previous window
// origin, its distance, the frame being processed) stays in device memory,
// so a whole sequence of frames is enqueued, or one captured step replayed
// per frame, without reading anything back.  The fallback decision
// of the learned search is taken on the device: when the best proposal is
// accepted, the exhaustive candidate list is filled with origins outside
// every frame, so the exhaustive scoring that follows finds no candidate
// inside and returns at once.
#include <algorithm>

#include "ih_internal.h"
#include "ih_lp.h"

namespace ih {

constexpr int32_t kFar = -(1 << 30);  // an origin outside every frame

// dst = frame st->frame of the stack (16-byte chunks, then the tail bytes).
__global__ void k_track_fetch(const uint8_t *__restrict__ stack, int64_t frame_bytes, int n_frames,
                              const ih_track_state *__restrict__ st, uint8_t *__restrict__ dst) {
  const int f = st->frame;
  if (f < 0 || f >= n_frames) return;
  const uint8_t *src = stack + (int64_t)f * frame_bytes;
  const int64_t n16 = frame_bytes >> 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
  for (int64_t i = (n16 << 4) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < frame_bytes; i += stride)
    dst[i] = src[i];
}

__global__ void k_track_prepare(ih_track_state *__restrict__ st, int win_h, int win_w, int32_t *__restrict__ base,
                                int32_t *__restrict__ center) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int32_t r = st->origin[0], c = st->origin[1];
  base[0] = r;
  base[1] = c;
  if (center) {
    center[0] = r + win_h / 2;
    center[1] = c + win_w / 2;
  }
  st->decision = -1;
  st->scored = 0;
}

// Accept the best proposal when its distance is within (1 + tau) times the
// previous frame's; otherwise list every offset for the exhaustive search.
__global__ void k_track_gate(ih_track_state *__restrict__ st, const int32_t *__restrict__ idx,
                             const float *__restrict__ kdist, const int32_t *__restrict__ kbest, int radius,
                             double tau, const int32_t *__restrict__ base, int32_t *__restrict__ exh) {
  const int n = 2 * radius + 1;
  const int b = kbest[0];
  const double d = b >= 0 ? (double)kdist[b] : (double)INFINITY;
  const bool accept = b >= 0 && d <= (1.0 + tau) * (double)st->dist;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    st->decision = accept ? idx[b] : -1;
    st->scored = accept ? 0 : n * n;
  }
  if (i < n * n) {
    exh[2 * i] = accept ? kFar : base[0] + i / n - radius;
    exh[2 * i + 1] = accept ? kFar : base[1] + i % n - radius;
  }
}

// Bounded form of the gate.  When the margin rule accepts the best proposal
// (distance d), every offset whose lower bound lb exceeds d by more than the
// rounding of both figures is dropped from the exhaustive list (set outside
// every frame) and the rest stay listed: the scoring of that list then
// returns the exhaustive search's own argmin and distance.  (lb is the
// pyramid distance with one level fewer: merging cells never raises a
// chi-square or L1 sum, so each level's sum is at least the coarser one's,
// and with Eq. 2.24's weights the distance of L + 1 levels exceeds that of L
// levels by a non-negative combination of those differences; a dropped
// offset therefore scores above d, which is at least the minimum.)
// Otherwise every offset is listed, as in the plain gate.
// st->decision = -2 (bounded) or -1 (fallback); st->scored counts the listed
// offsets (one block-wide count per block, then one atomic add).
__global__ __launch_bounds__(256) void k_track_gate_bounded(ih_track_state *__restrict__ st,
                                                             const float *__restrict__ kdist,
                                                             const int32_t *__restrict__ kbest, int radius,
                                                             double tau, const int32_t *__restrict__ base,
                                                             const float *__restrict__ lb,
                                                             int32_t *__restrict__ exh) {
  const int n = 2 * radius + 1;
  const int b = kbest[0];
  const double d = b >= 0 ? (double)kdist[b] : (double)INFINITY;
  const bool accept = b >= 0 && d <= (1.0 + tau) * (double)st->dist;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) st->decision = accept ? -2 : -1;
  bool listed = false;
  if (i < n * n) {
    // both figures carry at most a few FP32 roundings (relative 2^-22 each);
    // 2^-16 of slack keeps every offset whose true bound is <= d
    listed = !accept || !((double)lb[i] > d * (1.0 + 1.0 / 65536.0));
    exh[2 * i] = listed ? base[0] + i / n - radius : kFar;
    exh[2 * i + 1] = listed ? base[1] + i % n - radius : kFar;
  }
  const int cnt = __syncthreads_count(listed);
  if (threadIdx.x == 0 && cnt) atomicAdd(&st->scored, cnt);
}

__global__ void k_track_commit(ih_track_state *__restrict__ st, const float *__restrict__ kdist,
                               const int32_t *__restrict__ kbest, const float *__restrict__ edist,
                               const int32_t *__restrict__ ebest, int radius, int32_t *__restrict__ rec,
                               int n_rec) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int n = 2 * radius + 1;
  const int dec = st->decision;
  int32_t r = st->origin[0], c = st->origin[1];
  float d;
  int32_t fb;
  if (dec >= 0) {  // accepted proposal
    r += dec / n - radius;
    c += dec % n - radius;
    d = kdist[kbest[0]];
    fb = 0;
  } else {  // the exhaustive list decides: full (-1, a fallback) or bounded (-2)
    const int b = ebest[0];
    fb = dec == -1 ? 1 : 0;
    if (b >= 0) {
      r += b / n - radius;
      c += b % n - radius;
      d = edist[b];
    } else {
      d = INFINITY;
    }
  }
  st->origin[0] = r;
  st->origin[1] = c;
  st->dist = d;
  const int f = st->frame;
  if (f >= 0 && f < n_rec) {
    rec[5 * f] = r;
    rec[5 * f + 1] = c;
    rec[5 * f + 2] = __float_as_int(d);
    rec[5 * f + 3] = fb;
    rec[5 * f + 4] = st->scored;
  }
  st->frame = f + 1;
}

// Search region of the current frame: the (2 radius + win) x (2 radius + win)
// block of pixels that every candidate window around the previous origin can
// touch, shifted inside the frame.  region [C][rh][rw] gets those pixels;
// rbase [2] the previous origin in region coordinates, so that candidate
// origins rbase + offset address the region's integral histogram.  Every
// candidate window inside the frame lies inside the region, and every window
// that leaves the frame also leaves the region, so the search over the
// region's histogram equals the search over the frame's.
__global__ void k_track_region(const uint8_t *__restrict__ frame, int C, int H, int W,
                               const ih_track_state *__restrict__ st, int radius, int rh, int rw,
                               uint8_t *__restrict__ region, int32_t *__restrict__ rbase) {
  const int r0 = min(max(st->origin[0] - radius, 0), H - rh);
  const int c0 = min(max(st->origin[1] - radius, 0), W - rw);
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    rbase[0] = st->origin[0] - r0;
    rbase[1] = st->origin[1] - c0;
  }
  const int64_t n = (int64_t)C * rh * rw;
  for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ch = i / ((int64_t)rh * rw);
    const int rem = (int)(i - ch * rh * rw);
    const int y = rem / rw, x = rem - y * rw;
    region[i] = frame[(ch * H + r0 + y) * W + c0 + x];
  }
}

// Local refinement of the best candidate found so far (idx[kbest[0]],
// kdist[kbest[0]]): the origins of the (2q+1)^2 offsets around it, in
// row-major order, those outside the search range set outside every frame.
__global__ void k_track_refine_origins(const int32_t *__restrict__ idx, const int32_t *__restrict__ kbest, int q,
                                       int radius, const int32_t *__restrict__ base, int32_t *__restrict__ out) {
  const int m = 2 * q + 1, n = 2 * radius + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  const int b = kbest[0];
  int32_t r = kFar, c = kFar;
  if (b >= 0) {
    const int off = idx[b];
    const int oy = off / n - radius + i / m - q, ox = off % n - radius + i % m - q;
    if (oy >= -radius && oy <= radius && ox >= -radius && ox <= radius) {
      r = base[0] + oy;
      c = base[1] + ox;
    }
  }
  out[2 * i] = r;
  out[2 * i + 1] = c;
}

// Moves the best candidate to the neighbourhood's best (nbest, ndist) when
// that is smaller, or equal at a lower offset index (the exhaustive search's
// tie rule), and stores the result in slot 0: idx[0], kdist[0], kbest[0] = 0.
__global__ void k_track_refine_pick(int32_t *__restrict__ idx, float *__restrict__ kdist, int32_t *__restrict__ kbest,
                                    const float *__restrict__ ndist, const int32_t *__restrict__ nbest, int q,
                                    int radius) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int m = 2 * q + 1, n = 2 * radius + 1;
  const int b = kbest[0];
  if (b < 0) return;
  int off = idx[b];
  float d = kdist[b];
  const int nb = nbest[0];
  if (nb >= 0) {
    const int noff = off + (nb / m - q) * n + (nb % m - q);
    const float nd = ndist[nb];
    if (nd < d || (nd == d && noff < off)) {
      off = noff;
      d = nd;
    }
  }
  idx[0] = off;
  kdist[0] = d;
  kbest[0] = 0;
}

}  // namespace ih

using namespace ih;

extern "C" int ih_track_region(const void *frame, int32_t C, int32_t H, int32_t W, const ih_track_state *st,
                               int32_t radius, int32_t win_h, int32_t win_w, void *region, int32_t *rbase,
                               void *stream) {
  if (!frame || !st || !region || !rbase || C < 1 || H < 1 || W < 1 || radius < 0 || win_h < 1 || win_w < 1)
    return set_error(IH_ERR_INVALID_ARG, "bad track-region arguments");
  const int64_t rh = 2 * (int64_t)radius + win_h, rw = 2 * (int64_t)radius + win_w;
  if (rh > H || rw > W)
    return set_error(IH_ERR_RANGE, "search region %lldx%lld larger than the %dx%d frame", (long long)rh,
                     (long long)rw, H, W);
  const int64_t n = (int64_t)C * rh * rw;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_track_region, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), (const uint8_t *)frame,
                     C, H, W, st, radius, (int)rh, (int)rw, (uint8_t *)region, rbase);
  return hip_check(hipGetLastError(), "track region launch");
}

extern "C" int ih_track_refine_origins(const int32_t *idx, const int32_t *kbest, int32_t q, int32_t radius,
                                       const int32_t *base, int32_t *origins, void *stream) {
  if (!idx || !kbest || !base || !origins || q < 1 || q > 32 || radius < 0 || radius > 4096)
    return set_error(IH_ERR_INVALID_ARG, "bad track-refine arguments");
  const int m = 2 * q + 1;
  hipLaunchKernelGGL(k_track_refine_origins, dim3((m * m + 255) / 256), dim3(256), 0, as_stream(stream), idx, kbest,
                     q, radius, base, origins);
  return hip_check(hipGetLastError(), "track refine-origins launch");
}

extern "C" int ih_track_refine_pick(int32_t *idx, float *kdist, int32_t *kbest, const float *ndist,
                                    const int32_t *nbest, int32_t q, int32_t radius, void *stream) {
  if (!idx || !kdist || !kbest || !ndist || !nbest || q < 1 || q > 32 || radius < 0 || radius > 4096)
    return set_error(IH_ERR_INVALID_ARG, "bad track-refine arguments");
  hipLaunchKernelGGL(k_track_refine_pick, dim3(1), dim3(64), 0, as_stream(stream), idx, kdist, kbest, ndist, nbest,
                     q, radius);
  return hip_check(hipGetLastError(), "track refine-pick launch");
}

extern "C" int ih_track_fetch(const void *stack, int64_t frame_bytes, int32_t n_frames, const ih_track_state *st,
                              void *dst, void *stream) {
  if (!stack || !st || !dst || frame_bytes < 1 || n_frames < 1)
    return set_error(IH_ERR_INVALID_ARG, "bad track-fetch arguments");
  if (((uintptr_t)stack | (uintptr_t)dst | (uintptr_t)frame_bytes) & 15)
    return set_error(IH_ERR_INVALID_ARG, "stack, dst and frame_bytes must be multiples of 16 bytes");
  const int64_t n16 = frame_bytes >> 4;
  const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_track_fetch, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, as_stream(stream),
                     (const uint8_t *)stack, frame_bytes, n_frames, st, (uint8_t *)dst);
  return hip_check(hipGetLastError(), "track fetch launch");
}

extern "C" int ih_track_prepare(ih_track_state *st, int32_t win_h, int32_t win_w, int32_t *base, int32_t *center,
                                void *stream) {
  if (!st || !base || win_h < 1 || win_w < 1) return set_error(IH_ERR_INVALID_ARG, "bad track-prepare arguments");
  hipLaunchKernelGGL(k_track_prepare, dim3(1), dim3(64), 0, as_stream(stream), st, win_h, win_w, base, center);
  return hip_check(hipGetLastError(), "track prepare launch");
}

extern "C" int ih_track_gate(ih_track_state *st, const int32_t *idx, const float *kdist, const int32_t *kbest,
                             int32_t radius, double tau, const int32_t *base, int32_t *exh_origins, void *stream) {
  if (!st || !idx || !kdist || !kbest || !base || !exh_origins || radius < 0 || radius > 4096)
    return set_error(IH_ERR_INVALID_ARG, "bad track-gate arguments");
  const int nn = (2 * radius + 1) * (2 * radius + 1);
  hipLaunchKernelGGL(k_track_gate, dim3((nn + 255) / 256), dim3(256), 0, as_stream(stream), st, idx, kdist, kbest,
                     radius, tau, base, exh_origins);
  return hip_check(hipGetLastError(), "track gate launch");
}

extern "C" int ih_track_gate_bounded(ih_track_state *st, const float *kdist, const int32_t *kbest, int32_t radius,
                                     double tau, const int32_t *base, const float *lb, int32_t *exh_origins,
                                     void *stream) {
  if (!st || !kdist || !kbest || !base || !lb || !exh_origins || radius < 0 || radius > 4096)
    return set_error(IH_ERR_INVALID_ARG, "bad track-gate arguments");
  const int nn = (2 * radius + 1) * (2 * radius + 1);
  hipLaunchKernelGGL(k_track_gate_bounded, dim3((nn + 255) / 256), dim3(256), 0, as_stream(stream), st, kdist,
                     kbest, radius, tau, base, lb, exh_origins);
  return hip_check(hipGetLastError(), "track bounded-gate launch");
}

extern "C" int ih_track_commit(ih_track_state *st, const float *kdist, const int32_t *kbest, const float *exh_dist,
                               const int32_t *exh_best, int32_t radius, int32_t *rec, int32_t n_rec, void *stream) {
  if (!st || !exh_dist || !exh_best || !rec || radius < 0 || radius > 4096 || n_rec < 1)
    return set_error(IH_ERR_INVALID_ARG, "bad track-commit arguments");
  hipLaunchKernelGGL(k_track_commit, dim3(1), dim3(64), 0, as_stream(stream), st, kdist, kbest, exh_dist, exh_best,
                     radius, rec, n_rec);
  return hip_check(hipGetLastError(), "track commit launch");
}
