// Batched build + search of many uneven frames in one persistent launch.
//
// Work is cut into tickets in six phases, phase-major and frame-minor:
//   0 tile histograms, 1 carry scans, 2 write-out, 3 template descriptor,
//   4 candidate scoring (64 candidates per ticket), 5 best candidate.
// A fixed grid of resident workgroups takes tickets from an atomic counter in
// increasing order.  A ticket of phase k of frame f first waits until every
// ticket of the phase it depends on for the same frame has completed
// (per-frame, per-phase completion counters, released and acquired at device
// scope); because tickets are taken in order, everything a ticket waits on
// was taken earlier by a running workgroup, so every wait ends.  The bodies
// are the same device code as the stand-alone kernels.
#include "ih_build_dev.h"
#include "ih_match_dev.h"

namespace ih {

constexpr int NPH = 6;
constexpr int kBatchLds = 32 * 1024;  // LDS budget of the tile-histogram phase

struct FramePlan {
  Geom g;
  const void *img;
  int32_t *ih;
  int32_t bits, bc, gy, vec_ok;
  int64_t tiles;           // tiles of the grid (x channels)
  int64_t ws_off;          // word offset of this frame's carries in the carry area
  int64_t nA, nB;          // carry-scan job split
  int64_t cnt[NPH];        // tickets of this frame per phase
  int64_t start[NPH];      // first global ticket of this frame per phase
  const int32_t *tmpl_desc;
  int32_t *tmpl_out;
  int32_t tmpl_win[4];
  int32_t win_h, win_w;
  const int32_t *origins;
  int64_t n_cand;
  float *dist;
  int32_t *best;
};

struct BatchHeader {
  int32_t n, dtype, metric, lds;  // lds: dynamic LDS bytes of the persistent kernel
  int64_t phase_start[NPH + 1];
  int64_t counter_words;          // counters at the start of the workspace
  int64_t ws_words;
};

__device__ __forceinline__ int find_frame(const FramePlan *__restrict__ fr, int n, int ph, int64_t t) {
  int lo = 0, hi = n - 1;  // largest f with start[ph] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fr[mid].start[ph] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Bounded wait for a completion counter.  Every wait is for tickets taken
// earlier, so it ends; the bound only guarantees that no wave can spin
// forever should that invariant ever be broken: the wait then gives up,
// raises the batch's error flag and carries on.
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ void wait_count(uint32_t *c, int64_t need, uint32_t *err) {
  uint32_t spins = 0;
  while ((int64_t)__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (++spins >= kSpinLimit) {
      __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T>
__device__ __forceinline__ void final_dispatch(const FinalArgs &a, const Geom &g, int bx, int by) {
  const int wave = uniform(threadIdx.x >> 6);
#define IH_B(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) { final_body<T, C_, G_, false>(a, g, bx, by, wave, 4); return; }
  IH_B(1, 1) IH_B(1, 2) IH_B(1, 4) IH_B(1, 8)
  IH_B(2, 1) IH_B(2, 2) IH_B(2, 4) IH_B(2, 8)
  IH_B(4, 1) IH_B(4, 2) IH_B(4, 4) IH_B(4, 8)
#undef IH_B
}

__global__ void k_batch_reset(uint32_t *__restrict__ ws, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    ws[i] = 0;
}

template <typename T, int METRIC>
__global__ __launch_bounds__(256) void k_batch(const BatchHeader *__restrict__ hdr, const FramePlan *__restrict__ fr,
                                               uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t s_ticket;
  const int n = hdr->n;
  const int64_t total = hdr->phase_start[NPH];
  uint32_t *ticket = ws;
  uint32_t *done = ws + 1;
  uint32_t *err = ws + 1 + NPH * n;
  uint32_t *carry = ws + hdr->counter_words;
  for (;;) {
    if (threadIdx.x == 0)
      s_ticket = (int64_t)__hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t t = s_ticket;
    if (t >= total) break;
    int ph = 0;
    while (t >= hdr->phase_start[ph + 1]) ++ph;
    const int f = find_frame(fr, n, ph, t);
    const FramePlan &F = fr[f];
    const int64_t u = t - F.start[ph];
    if (threadIdx.x == 0) {
      if (ph >= 1 && ph <= 3) wait_count(&done[(ph - 1) * n + f], F.cnt[ph - 1], err);
      if (ph == 4) {
        wait_count(&done[2 * n + f], F.cnt[2], err);
        wait_count(&done[3 * n + f], F.cnt[3], err);
      }
      if (ph == 5) wait_count(&done[4 * n + f], F.cnt[4], err);
    }
    __syncthreads();
    uint32_t *fws = carry + F.ws_off;
    const Geom &g = F.g;
    switch (ph) {
      case 0:
        tile_hist_body<T>(reinterpret_cast<const T *>(F.img), g, F.bits, F.bc, fws, (int)u, lds);
        break;
      case 1:
        carry_scan_body(g, F.nA, F.nB, fws, u);
        break;
      case 2: {
        const FinalArgs a{F.img, F.ih, nullptr, nullptr, fws, F.bits, F.vec_ok};
        final_dispatch<T>(a, g, (int)(u % F.tiles), (int)(u / F.tiles));
        break;
      }
      case 3:
        for (int p = threadIdx.x; p < g.P; p += blockDim.x)
          pyramid_cells<3>(F.ih, g.P, g.H, g.W, IH_BHW, F.tmpl_win, p, F.tmpl_out + p);
        break;
      case 4: {
        const int32_t *tm = F.tmpl_desc ? F.tmpl_desc : F.tmpl_out;
        match_body<3, METRIC>(F.ih, g.P, g.H, g.W, tm, F.win_h, F.win_w, F.origins, F.n_cand, F.dist, u,
                              reinterpret_cast<double *>(lds), reinterpret_cast<long long *>(lds) + 64 * kMatchWaves);
        break;
      }
      default:
        argbest_body<METRIC == IH_PMK>(F.dist, F.n_cand, F.best, reinterpret_cast<float *>(lds),
                                       reinterpret_cast<int64_t *>(lds) + 256);
        break;
    }
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[ph * n + f], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

typedef void (*batch_fn)(const BatchHeader *, const FramePlan *, uint32_t *);

template <typename T>
static batch_fn pick_batch_t(int metric) {
  if (metric == IH_CHI2) return &k_batch<T, IH_CHI2>;
  if (metric == IH_L1) return &k_batch<T, IH_L1>;
  return &k_batch<T, IH_PMK>;
}

static batch_fn pick_batch(int dtype, int metric) {
  return dtype == IH_U8 ? pick_batch_t<uint8_t>(metric) : pick_batch_t<uint16_t>(metric);
}

static size_t a64(size_t w) { return (w + 63) & ~(size_t)63; }

}  // namespace ih

using namespace ih;

extern "C" size_t ih_batch_plan_bytes(int32_t n) {
  return n < 1 ? 0 : sizeof(BatchHeader) + (size_t)n * sizeof(FramePlan);
}

extern "C" int ih_batch_plan(const ih_frame *frames, int32_t n, int32_t dtype, int32_t metric, void *plan,
                             size_t plan_bytes, size_t *ws_bytes) {
  if (n < 1 || !frames || !plan || !ws_bytes) return set_error(IH_ERR_INVALID_ARG, "frames, plan, ws_bytes and n >= 1");
  if (plan_bytes < ih_batch_plan_bytes(n)) return set_error(IH_ERR_INVALID_ARG, "plan buffer too small");
  if (dtype != IH_U8 && dtype != IH_U16) return set_error(IH_ERR_INVALID_ARG, "dtype %d unknown", dtype);
  if (metric != IH_CHI2 && metric != IH_L1 && metric != IH_PMK)
    return set_error(IH_ERR_INVALID_ARG, "metric %d unknown", metric);
  BatchHeader *h = reinterpret_cast<BatchHeader *>(plan);
  FramePlan *fp = reinterpret_cast<FramePlan *>(h + 1);
  const int maxbits = dtype == IH_U8 ? 8 : 16;
  size_t carry = 0, lds = (size_t)kMatchWaves * 64 * 16;  // match partials: waves x 64 x (8 + 8) bytes
  if (lds < 256 * 16) lds = 256 * 16;                     // best-candidate reduction: 256 x (4 + 8), 8-aligned
  for (int f = 0; f < n; ++f) {
    const ih_frame &F = frames[f];
    FramePlan &P = fp[f];
    memset(&P, 0, sizeof P);
    if (!F.img || !F.ih) return set_error(IH_ERR_INVALID_ARG, "frame %d: img and ih must be non-NULL", f);
    if (F.value_bits < 1 || F.value_bits > maxbits)
      return set_error(IH_ERR_INVALID_ARG, "frame %d: value_bits %d outside 1..%d", f, F.value_bits, maxbits);
    if (F.bins > (1 << F.value_bits)) return set_error(IH_ERR_INVALID_ARG, "frame %d: bins exceed 2^value_bits", f);
    int e = make_geom(F.H, F.W, F.C, F.bins, 0, IH_BHW, F.tile.tile_h ? &F.tile : nullptr, &P.g);
    if (e) return set_error(e, "frame %d: %s", f, ih_last_error());
    if (P.g.PG > 8) return set_error(IH_ERR_UNSUPPORTED, "frame %d: planes_per_wave %d > 8 in a batch", f, P.g.PG);
    size_t l;
    if ((e = pick_bc(P.g, kBatchLds, &P.bc, &l))) return set_error(e, "frame %d: %s", f, ih_last_error());
    if (l > lds) lds = l;
    P.img = F.img;
    P.ih = F.ih;
    P.bits = F.value_bits;
    P.vec_ok = ((uintptr_t)F.ih % 16 == 0 && F.W % P.g.CPL == 0) ? 1 : 0;
    P.tiles = (int64_t)P.g.nTR * P.g.nTC * F.C;
    P.ws_off = (int64_t)carry;
    carry += a64(P.g.words);
    P.nA = ((int64_t)P.g.P * F.W + 255) / 256;
    P.nB = ((int64_t)F.C * F.H * F.bins + 255) / 256;
    const int groups = (F.bins + P.g.PG - 1) / P.g.PG;
    P.gy = (groups + 3) / 4;
    P.cnt[0] = P.tiles;
    P.cnt[1] = P.nA + P.nB + P.g.P;
    P.cnt[2] = P.tiles * P.gy;
    if (F.n_cand < 0) return set_error(IH_ERR_INVALID_ARG, "frame %d: n_cand < 0", f);
    if (F.n_cand > 0) {
      if (!F.origins || !F.dist || !F.best) return set_error(IH_ERR_INVALID_ARG, "frame %d: NULL search buffer", f);
      if (F.win_h < 1 || F.win_w < 1) return set_error(IH_ERR_INVALID_ARG, "frame %d: window must be positive", f);
      if (F.n_cand >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "frame %d: too many candidates", f);
      if (!F.tmpl_desc && !F.tmpl_out)
        return set_error(IH_ERR_INVALID_ARG, "frame %d: need tmpl_desc or tmpl_out", f);
      P.tmpl_desc = F.tmpl_desc;
      P.tmpl_out = F.tmpl_out;
      for (int k = 0; k < 4; ++k) P.tmpl_win[k] = F.tmpl_win[k];
      P.win_h = F.win_h;
      P.win_w = F.win_w;
      P.origins = F.origins;
      P.n_cand = F.n_cand;
      P.dist = F.dist;
      P.best = F.best;
      P.cnt[3] = F.tmpl_desc ? 0 : 1;
      P.cnt[4] = (F.n_cand + 63) / 64;
      P.cnt[5] = 1;
    }
  }
  int64_t s = 0;
  for (int ph = 0; ph < NPH; ++ph) {
    h->phase_start[ph] = s;
    for (int f = 0; f < n; ++f) {
      fp[f].start[ph] = s;
      s += fp[f].cnt[ph];
    }
  }
  h->phase_start[NPH] = s;
  if (s >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "batch of %lld tickets too large", (long long)s);
  h->n = n;
  h->dtype = dtype;
  h->metric = metric;
  h->lds = (int32_t)lds;
  h->counter_words = (int64_t)a64(2 + (size_t)NPH * n);  // ticket, done[NPH][n], error flag
  h->ws_words = h->counter_words + (int64_t)carry;
  *ws_bytes = (size_t)h->ws_words * 4;
  return IH_OK;
}

extern "C" int ih_build_batch(const void *plan_host, const void *plan_dev, void *ws, size_t ws_bytes, void *stream) {
  if (!plan_host || !plan_dev) return set_error(IH_ERR_INVALID_ARG, "plan_host and plan_dev must be non-NULL");
  const BatchHeader *h = reinterpret_cast<const BatchHeader *>(plan_host);
  if (h->n < 1 || (h->dtype != IH_U8 && h->dtype != IH_U16))
    return set_error(IH_ERR_INVALID_ARG, "plan not initialised by ih_batch_plan");
  if (!ws || ws_bytes < (size_t)h->ws_words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %lld bytes needed", (long long)h->ws_words * 4);
  hipStream_t s = as_stream(stream);
  batch_fn fn = pick_batch(h->dtype, h->metric);
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    int e;
    if ((e = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return e;
    if ((e = hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties"))) return e;
    cus = prop.multiProcessorCount;
  }
  int per_cu = 0;
  int e = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, h->lds), "occupancy");
  if (e) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t total = h->phase_start[NPH];
  int64_t blocks = (int64_t)per_cu * cus;
  if (blocks > total) blocks = total > 0 ? total : 1;
  uint32_t *w32 = reinterpret_cast<uint32_t *>(ws);
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, w32, h->counter_words);
  if ((e = hip_check(hipGetLastError(), "batch reset launch"))) return e;
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(plan_dev);
  const FramePlan *fd = reinterpret_cast<const FramePlan *>(hd + 1);
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), h->lds, s, hd, fd, w32);
  return hip_check(hipGetLastError(), "batch launch");
}

extern "C" size_t ih_batch_error_offset(int32_t n) { return n < 1 ? 0 : (size_t)(1 + NPH * (size_t)n) * 4; }
