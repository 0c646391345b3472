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
  if (i == 0) st->decision = accept ? idx[b] : -1;
  if (i < n * n) {
    exh[2 * i] = accept ? kFar : base[0] + i / n - radius;
    exh[2 * i + 1] = accept ? kFar : base[1] + i % n - radius;
  }
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
  if (dec >= 0) {
    r += dec / n - radius;
    c += dec % n - radius;
    d = kdist[kbest[0]];
    fb = 0;
  } else {
    const int b = ebest[0];
    fb = 1;
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
    rec[4 * f] = r;
    rec[4 * f + 1] = c;
    rec[4 * f + 2] = __float_as_int(d);
    rec[4 * f + 3] = fb;
  }
  st->frame = f + 1;
}

}  // namespace ih

using namespace ih;

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

extern "C" int ih_track_commit(ih_track_state *st, const float *kdist, const int32_t *kbest, const float *exh_dist,
                               const int32_t *exh_best, int32_t radius, int32_t *rec, int32_t n_rec, void *stream) {
  if (!st || !exh_dist || !exh_best || !rec || radius < 0 || radius > 4096 || n_rec < 1)
    return set_error(IH_ERR_INVALID_ARG, "bad track-commit arguments");
  hipLaunchKernelGGL(k_track_commit, dim3(1), dim3(64), 0, as_stream(stream), st, kdist, kbest, exh_dist, exh_best,
                     radius, rec, n_rec);
  return hip_check(hipGetLastError(), "track commit launch");
}
