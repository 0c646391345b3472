// Device side of the batched build + search: the plan structures, the unit
// bodies of the six phases and the kernels that run them (one kernel per
// phase, or one cooperative kernel for all).  Included by the host code that
// launches the phased kernels and by the translation unit that holds the
// cooperative kernels, so that the two compile in parallel.
#pragma once
#include "ih_build_dev.h"
#include "ih_match_dev.h"

#include <hip/hip_cooperative_groups.h>

namespace ih {

constexpr int NPH = 6;
constexpr int kLayStrip = 2;    // write-out class of the frames that take the strip write-out
constexpr int kLayStreams = 3;  // write-out class of planes-innermost frames split into column streams
constexpr int kBatchLds = 32 * 1024;  // LDS budget of the tile-histogram phase
#ifndef IH_BATCH_BHW_TH
#define IH_BATCH_BHW_TH 64
#define IH_BATCH_BHW_TW 64
#define IH_BATCH_HWB_TH 64
#define IH_BATCH_HWB_TW 32
#endif

struct FramePlan {
  Geom g;
  const void *img;
  int32_t *ih;
  int32_t bits, bc, gy, vec_ok;
  int64_t tiles;           // tiles of the grid (x channels)
  int64_t ws_off;          // word offset of this frame's carries in the workspace
  int64_t nA, nB;          // carry-scan job split
  int64_t cnt[NPH];        // units of this frame per phase
  int64_t start[NPH];      // first unit of this frame in the phase's numbering
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
  int32_t n, dtype, metric, lds;  // lds: dynamic LDS bytes of the cooperative kernel (all phases)
  int32_t lds_ph[NPH];            // dynamic LDS bytes of each phase's own kernel (phased mode)
  int32_t layouts;                // bit l set: some frame uses layout l
  int32_t wclasses;               // bit c set: some frame's write-out is of class c (batch_wclass)
  int32_t lds_strip;              // dynamic LDS bytes of the strip write-out kernel
  int64_t phase_start[NPH + 1];   // unit numbering: phase-major, frame-minor
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

// Strip write-out (bin-major plain counts with rows not 64-byte aligned):
// unit ux of the frame's strips, plane group grp, this wave's LDS ring.
template <typename T>
__device__ __forceinline__ void strip_dispatch(const FinalArgs &a, const Geom &g, int64_t ux, int grp, uint32_t *ring) {
#define IH_S(C_, G_) \
  if (g.CPL == C_ && g.PG == G_) { final_strip_body<T, C_, G_>(a, g, ux, grp, ring); return; }
  IH_S(1, 1) IH_S(1, 2) IH_S(1, 4) IH_S(1, 8)
  IH_S(2, 1) IH_S(2, 2) IH_S(2, 4) IH_S(2, 8)
  IH_S(4, 1) IH_S(4, 2) IH_S(4, 4) IH_S(4, 8)
#undef IH_S
}

// Planes-innermost write-out in a batch: four wave units per workgroup unit;
// frames of at most 64 planes stage each tile row in the wave's LDS slice.
// Write-out class of a frame: its layout, or kLayStrip (bin-major strip
// write-out) or kLayStreams (planes-innermost frames of at most 32 planes
// and 32-column tiles, split into column streams).  Each class has its own
// write-out kernel, compiled alone (its own registers, hence occupancy).
__host__ __device__ inline int batch_wclass(const Geom &g) {
  if (g.strip) return kLayStrip;
  if (g.layout == IH_HWB && g.P <= 32 && g.TW <= 32) return kLayStreams;
  return g.layout;
}

template <typename T, int LAY = -1>
__device__ __forceinline__ void final_hwb_batch(const FinalArgs &a, const Geom &g, int64_t u, uint32_t *lds) {
  const int wave = uniform((int)(threadIdx.x >> 6));
  const int64_t wu = u * 4 + wave;
  uint32_t *slice = lds + wave * g.TW * 64;
  if constexpr (LAY == -1 || LAY == kLayStreams) {
    if (batch_wclass(g) == kLayStreams) {
      // few planes: the wave splits into column streams (lanes over stream x plane)
      if (g.P <= 8) {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 8>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 8>(a, g, wu, slice);
      } else if (g.P <= 16) {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 4>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 4>(a, g, wu, slice);
      } else {
        if (g.TW == 16) final_hwb_wave_streams_body<T, 16, 2>(a, g, wu, slice);
        else final_hwb_wave_streams_body<T, 32, 2>(a, g, wu, slice);
      }
      return;
    }
  }
  if constexpr (LAY != kLayStreams) {
    if (g.P <= 64 && g.TW <= 32) {
      if (g.TW == 16) final_hwb_wave_staged_body<T, 16>(a, g, wu, slice);
      else final_hwb_wave_staged_body<T, 32>(a, g, wu, slice);
    } else {
      if (g.TW == 16) final_hwb_body<T, 16, false>(a, g, wu);
      else if (g.TW == 32) final_hwb_body<T, 32, false>(a, g, wu);
      else final_hwb_body<T, 64, false>(a, g, wu);
    }
  }
}

// One unit of phase ph: the u-th unit of frame F.
template <typename T, int METRIC, int LAY = -1>
__device__ __forceinline__ void run_unit(const FramePlan &F, int ph, int64_t u, uint32_t *ws, uint32_t *lds) {
  uint32_t *fws = ws + F.ws_off;
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
      if constexpr (LAY == -1 || LAY == IH_HWB || LAY == kLayStreams) {
        if (g.layout == IH_HWB) { final_hwb_batch<T, LAY>(a, g, u, lds); break; }
      }
      if constexpr (LAY == -1 || LAY == kLayStrip) {
        if (g.strip) {
          const int wave = uniform((int)(threadIdx.x >> 6));
          const int64_t X = strip_units(g);
          strip_dispatch<T>(a, g, u % X, (int)(u / X) * 4 + wave, lds + (size_t)wave * (strip_lds_wave(g) / 4));
          break;
        }
      }
      if constexpr (LAY == -1 || LAY == IH_BHW) final_dispatch<T>(a, g, (int)(u % F.tiles), (int)(u / F.tiles));
      break;
    }
    case 3:
      for (int p = threadIdx.x; p < g.P; p += blockDim.x)
        pyramid_cells<3>(F.ih, g.P, g.H, g.W, g.layout, F.tmpl_win, p, F.tmpl_out + p);
      break;
    case 4: {
      const int32_t *tm = F.tmpl_desc ? F.tmpl_desc : F.tmpl_out;
      if constexpr (LAY != IH_BHW) {
        if (g.layout == IH_HWB) {
          match_hwb_body<3, METRIC>(F.ih, g.P, g.H, g.W, tm, F.win_h, F.win_w, F.origins, F.n_cand, F.dist,
                                    u * 4 + uniform((int)(threadIdx.x >> 6)));
          break;
        }
      }
      if constexpr (LAY != IH_HWB)
        match_body<3, METRIC>(F.ih, g.P, g.H, g.W, tm, F.win_h, F.win_w, F.origins, F.n_cand, F.dist, u,
                              reinterpret_cast<double *>(lds), reinterpret_cast<long long *>(lds) + 64 * kMatchWaves);
      break;
    }
    default:
      argbest_body<METRIC == IH_PMK>(F.dist, F.n_cand, F.best, reinterpret_cast<float *>(lds),
                                     reinterpret_cast<int64_t *>(lds) + 256);
      break;
  }
}

// All units of phase ph, grid-stride.  The unit of a workgroup iteration is
// uniform across the workgroup, so the bodies' barriers are reached by all.
// LAY >= 0 restricts the phase to frames of that layout (the others' units
// are skipped, uniformly per workgroup); in the write-out phase kLayStrip
// takes the bin-major frames of the strip write-out and IH_BHW the others.
template <typename T, int METRIC, int LAY = -1>
__device__ __forceinline__ void run_phase(const BatchHeader *__restrict__ hdr, const FramePlan *__restrict__ fr,
                                          uint32_t *__restrict__ ws, int ph, uint32_t *lds) {
  const int n = hdr->n;
  const int64_t end = hdr->phase_start[ph + 1];
  for (int64_t t = hdr->phase_start[ph] + blockIdx.x; t < end; t += gridDim.x) {
    const int f = find_frame(fr, n, ph, t);
    if (LAY >= 0 && (ph == 2 ? batch_wclass(fr[f].g) : fr[f].g.layout) != LAY) continue;
    run_unit<T, METRIC, LAY>(fr[f], ph, t - fr[f].start[ph], ws, lds);
    __syncthreads();
  }
}

// Phased mode: one kernel per phase, so that each phase is compiled alone
// (its own register count and LDS request, hence its own occupancy).
template <typename T, int METRIC, int PH, int LAY>
__global__ __launch_bounds__(256) void k_batch_phase(const BatchHeader *__restrict__ hdr,
                                                     const FramePlan *__restrict__ fr, uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  run_phase<T, METRIC, LAY>(hdr, fr, ws, PH, lds);
}

template <typename T, int METRIC>
__global__ __launch_bounds__(256) void k_batch_coop(const BatchHeader *__restrict__ hdr,
                                                    const FramePlan *__restrict__ fr, uint32_t *__restrict__ ws) {
  extern __shared__ uint32_t lds[];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int ph = 0; ph < NPH; ++ph) {
    if (hdr->phase_start[ph + 1] == hdr->phase_start[ph]) continue;  // the same for every workgroup
    run_phase<T, METRIC>(hdr, fr, ws, ph, lds);
    grid.sync();
  }
}

typedef void (*phase_fn)(const BatchHeader *, const FramePlan *, uint32_t *);
typedef void (*coop_fn)(const BatchHeader *, const FramePlan *, uint32_t *);


// The cooperative kernel for a metric, u8 or u16 pixels: instantiated in a
// translation unit per pixel type (each kernel holds every phase's bodies,
// so the two compile in parallel).
template <typename T>
coop_fn pick_coop_t(int metric) {
  if (metric == IH_CHI2) return &k_batch_coop<T, IH_CHI2>;
  if (metric == IH_L1) return &k_batch_coop<T, IH_L1>;
  return &k_batch_coop<T, IH_PMK>;
}
coop_fn pick_coop_u8(int metric);
coop_fn pick_coop_u16(int metric);

}  // namespace ih
