// Batched build + search of many uneven frames.
//
// Work is cut into units in six phases: 0 tile histograms, 1 carry scans,
// 2 write-out, 3 template descriptor, 4 candidate scoring (64 candidates per
// unit), 5 best candidate.  A phase of a frame depends only on earlier
// phases of the same frame.  Two ways to run a plan:
//   phased:      one launch per non-empty phase, each a grid-stride loop over
//                that phase's units of all frames (kernel boundaries order the
//                phases);
//   cooperative: one cooperative launch whose resident workgroups loop over
//                the units of each phase in turn, separated by the runtime's
//                grid-wide barrier.
// The unit bodies are the same device code as the stand-alone kernels.
#include "ih_batch_dev.h"

#include <mutex>

namespace ih {

// pf[ph][l]: the phase-ph kernel for frames of layout l (phases 2 and 4 have
// one kernel per layout, phase 2 a third for the strip write-out; the others
// serve every frame, entry [ph][0]).
template <typename T, int METRIC>
static void pick_m(phase_fn (*pf)[4]) {
  // phases 0-3 do not depend on the metric: one instance serves all three
  pf[0][0] = &k_batch_phase<T, IH_CHI2, 0, -1>;
  pf[1][0] = &k_batch_phase<T, IH_CHI2, 1, -1>;
  pf[2][0] = &k_batch_phase<T, IH_CHI2, 2, IH_BHW>;
  pf[2][1] = &k_batch_phase<T, IH_CHI2, 2, IH_HWB>;
  pf[2][2] = &k_batch_phase<T, IH_CHI2, 2, kLayStrip>;
  pf[2][3] = &k_batch_phase<T, IH_CHI2, 2, kLayStreams>;
  pf[3][0] = &k_batch_phase<T, IH_CHI2, 3, -1>;
  pf[4][0] = &k_batch_phase<T, METRIC, 4, IH_BHW>;
  pf[4][1] = &k_batch_phase<T, METRIC, 4, IH_HWB>;
  pf[5][0] = &k_batch_phase<T, METRIC, 5, -1>;
}

template <typename T>
static void pick_t(int metric, phase_fn (*pf)[4]) {
  if (metric == IH_CHI2) pick_m<T, IH_CHI2>(pf);
  else if (metric == IH_L1) pick_m<T, IH_L1>(pf);
  else pick_m<T, IH_PMK>(pf);
}

static size_t a64(size_t w) { return (w + 63) & ~(size_t)63; }

// Auxiliary streams (default priority) and events that let the write-out
// classes of a phased batch run as parallel branches of the caller's stream;
// created once per device, outside stream capture, and kept until the process
// ends.  The mutex makes each fork-launch-join sequence atomic with respect
// to other host threads, which share these events.
#ifndef IH_BATCH_BRANCHES
#define IH_BATCH_BRANCHES 2  // 0: none; 1: write-out classes only; 2: also the scoring layouts
#endif
constexpr int kAuxDevs = 64, kAux = 3;
struct AuxStreams {
  bool ok, failed;
  hipStream_t s[kAux];
  hipEvent_t fork, join[kAux];
};
static AuxStreams g_aux[kAuxDevs];
static std::mutex g_aux_mu;

// Returns the device's auxiliary streams, creating them unless the caller's
// stream is being captured; nullptr when they are not available (the write-out
// classes then run one after another on the caller's stream).  Call with
// g_aux_mu held.
static const AuxStreams *aux_streams(int dev, bool capturing) {
  if (dev < 0 || dev >= kAuxDevs) return nullptr;
  AuxStreams &x = g_aux[dev];
  if (x.ok) return &x;
  if (x.failed || capturing) return nullptr;
  x.failed = true;  // until every object below exists
  for (int i = 0; i < kAux; ++i)
    if (hipStreamCreateWithFlags(&x.s[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
  for (int i = 0; i < kAux; ++i)
    if (hipEventCreateWithFlags(&x.join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
  x.failed = false;
  x.ok = true;
  return &x;
}

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
  size_t lph[NPH] = {0, 0, 0, 0, 0, 256 * 16};
  size_t lds_strip = 0;
  for (int f = 0; f < n; ++f) {
    const ih_frame &F = frames[f];
    FramePlan &P = fp[f];
    memset(&P, 0, sizeof P);
    if (!F.img || !F.ih) return set_error(IH_ERR_INVALID_ARG, "frame %d: img and ih must be non-NULL", f);
    if (F.value_bits < 1 || F.value_bits > maxbits)
      return set_error(IH_ERR_INVALID_ARG, "frame %d: value_bits %d outside 1..%d", f, F.value_bits, maxbits);
    if (F.bins > (1 << F.value_bits)) return set_error(IH_ERR_INVALID_ARG, "frame %d: bins exceed 2^value_bits", f);
    if (F.layout != IH_BHW && F.layout != IH_HWB)
      return set_error(IH_ERR_INVALID_ARG, "frame %d: layout %d unknown", f, F.layout);
    if (F.tile.passes == IH_PASSES_ONE)
      return set_error(IH_ERR_UNSUPPORTED, "frame %d: batches build in three passes", f);
    const bool hwb = F.layout == IH_HWB;
    // without a tile shape, batch defaults: many frames already fill the GPU,
    // so tiles are taller than the single-frame heuristic's (fewer, longer units)
    ih_tile_cfg dflt;
    if (hwb) dflt = ih_tile_cfg{IH_BATCH_HWB_TH, IH_BATCH_HWB_TW, 64};
    else dflt = ih_tile_cfg{IH_BATCH_BHW_TH, IH_BATCH_BHW_TW, F.bins >= 2 ? 2 : 1};
    int e = make_geom(F.H, F.W, F.C, F.bins, 0, F.layout, F.tile.tile_h ? &F.tile : &dflt, &P.g);
    if (e) return set_error(e, "frame %d: %s", f, ih_last_error());
    if (!hwb && P.g.PG > 8)
      return set_error(IH_ERR_UNSUPPORTED, "frame %d: planes_per_wave %d > 8 in a batch", f, P.g.PG);
    size_t l;
    P.g.c16 = F.H < 65536 && F.W < 65536;  // count carries fit 16 bits
    P.g.strip = use_strip(P.g, F.ih);
    if ((e = pick_bc(P.g, kBatchLds, &P.bc, &l))) return set_error(e, "frame %d: %s", f, ih_last_error());
    if (tile_fast(P.g)) l = tile_fast_lds(P.g);
    if (l > lds) lds = l;
    if (l > lph[0]) lph[0] = l;
    P.img = F.img;
    P.ih = F.ih;
    P.bits = F.value_bits;
    P.vec_ok = ((uintptr_t)F.ih % 16 == 0 && F.W % P.g.CPL == 0) ? 1 : 0;
    if (hwb && P.g.P <= 64 && P.g.TW <= 32) {
      const size_t slices = (size_t)4 * P.g.TW * 64 * 4;  // four waves' staged row segments
      if (slices > lds) lds = slices;
      if (slices > lph[2]) lph[2] = slices;
    }
    if (!hwb && F.n_cand > 0 && lph[4] < (size_t)kMatchWaves * 64 * 16) lph[4] = (size_t)kMatchWaves * 64 * 16;
    P.tiles = (int64_t)P.g.nTR * P.g.nTC * F.C;
    P.ws_off = (int64_t)carry;
    carry += a64(P.g.words);
    P.nA = (carry_threads_a(P.g) + 255) / 256;
    P.nB = (carry_threads_b(P.g) + 255) / 256;
    const int groups = (F.bins + P.g.PG - 1) / P.g.PG;
    P.gy = (groups + 3) / 4;
    P.cnt[0] = P.tiles;
    P.cnt[1] = P.nA + P.nB + P.g.P;
    P.cnt[2] = hwb ? ((int64_t)P.g.nTR * P.g.nTC * ((P.g.P + 63) / 64) + 3) / 4
                   : (P.g.strip ? strip_units(P.g) : P.tiles) * P.gy;
    if (P.g.strip) {
      const size_t rings = 4 * strip_lds_wave(P.g);  // four waves' LDS rings
      if (rings > lds) lds = rings;
      if (rings > lds_strip) lds_strip = rings;
    }
    if (F.n_cand < 0) return set_error(IH_ERR_INVALID_ARG, "frame %d: n_cand < 0", f);
    if (F.n_cand > 0) {
      if (!F.origins || !F.dist || !F.best) return set_error(IH_ERR_INVALID_ARG, "frame %d: NULL search buffer", f);
      if (F.win_h < 1 || F.win_w < 1) return set_error(IH_ERR_INVALID_ARG, "frame %d: window must be positive", f);
      if (F.n_cand >= ((int64_t)1 << 31)) return set_error(IH_ERR_RANGE, "frame %d: too many candidates", f);
      if (hwb && (int64_t)F.W * P.g.P > 0xffffffffLL)
        return set_error(IH_ERR_RANGE, "frame %d: W*P above 2^32-1 planes-innermost", f);
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
      P.cnt[4] = hwb ? (F.n_cand + 3) / 4 : (F.n_cand + 63) / 64;
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
  if (s >= ((int64_t)1 << 40)) return set_error(IH_ERR_RANGE, "batch of %lld units too large", (long long)s);
  h->n = n;
  h->dtype = dtype;
  h->metric = metric;
  h->lds = (int32_t)lds;
  for (int ph = 0; ph < NPH; ++ph) h->lds_ph[ph] = (int32_t)lph[ph];
  h->layouts = 0;
  h->wclasses = 0;
  for (int f = 0; f < n; ++f) {
    h->layouts |= 1 << fp[f].g.layout;
    h->wclasses |= 1 << batch_wclass(fp[f].g);
  }
  h->lds_strip = (int32_t)lds_strip;
  h->ws_words = carry > 0 ? (int64_t)carry : 64;
  *ws_bytes = (size_t)h->ws_words * 4;
  return IH_OK;
}

extern "C" int ih_build_batch(const void *plan_host, const void *plan_dev, void *ws, size_t ws_bytes, int32_t mode,
                              void *stream) {
  if (!plan_host || !plan_dev) return set_error(IH_ERR_INVALID_ARG, "plan_host and plan_dev must be non-NULL");
  const BatchHeader *h = reinterpret_cast<const BatchHeader *>(plan_host);
  if (h->n < 1 || (h->dtype != IH_U8 && h->dtype != IH_U16))
    return set_error(IH_ERR_INVALID_ARG, "plan not initialised by ih_batch_plan");
  if (mode != IH_BATCH_PHASED && mode != IH_BATCH_COOPERATIVE)
    return set_error(IH_ERR_INVALID_ARG, "batch mode %d unknown", mode);
  if (!ws || ws_bytes < (size_t)h->ws_words * 4)
    return set_error(IH_ERR_WORKSPACE, "workspace of %lld bytes needed", (long long)h->ws_words * 4);
  hipStream_t s = as_stream(stream);
  phase_fn pf[NPH][4] = {};
  if (h->dtype == IH_U8) pick_t<uint8_t>(h->metric, pf);
  else pick_t<uint16_t>(h->metric, pf);
  const coop_fn cf = h->dtype == IH_U8 ? pick_coop_u8(h->metric) : pick_coop_u16(h->metric);
  int dev = 0, e;
  if ((e = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return e;
  int cus = 0;
  if ((e = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count"))) return e;
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(plan_dev);
  const FramePlan *fd = reinterpret_cast<const FramePlan *>(hd + 1);
  uint32_t *w32 = reinterpret_cast<uint32_t *>(ws);
  int per_cu = 0;
  if (mode == IH_BATCH_PHASED) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((e = hip_check(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing"))) return e;
    int nclass = 0, nlay = 0;
    for (int l = 0; l < 4; ++l) {
      nclass += (h->wclasses >> l) & 1;
      nlay += (h->layouts >> l) & 1;
    }
    for (int ph = 0; ph < NPH; ++ph) {
      const int64_t units = h->phase_start[ph + 1] - h->phase_start[ph];
      if (units == 0) continue;
      // several write-out classes (or scoring layouts): the first on the
      // caller's stream, the others on auxiliary streams forked after the
      // previous phase and joined before the next (they write disjoint frames)
      std::unique_lock<std::mutex> lk(g_aux_mu, std::defer_lock);
      const AuxStreams *ax = nullptr;
      if ((IH_BATCH_BRANCHES >= 1 && ph == 2 && nclass > 1) || (IH_BATCH_BRANCHES >= 2 && ph == 4 && nlay > 1)) {
        lk.lock();
        ax = aux_streams(dev, cs != hipStreamCaptureStatusNone);
        if (ax && (e = hip_check(hipEventRecord(ax->fork, s), "fork event"))) return e;
      }
      int branch = 0;
      for (int l = 0; l < 4; ++l) {
        const bool split = pf[ph][1] != nullptr;
        if (!split && l > 0) break;
        phase_fn k = pf[ph][l];
        // the write-out phase runs one kernel per write-out class present, the
        // scoring phase one per layout
        const int present = ph == 2 ? h->wclasses : h->layouts;
        if (!k || (split && !(present & (1 << l)))) continue;
        const int lds_k = l == 2 ? h->lds_strip : h->lds_ph[ph];
        if ((e = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds_k), "occupancy")))
          return e;
        if (per_cu < 1) return set_error(IH_ERR_UNSUPPORTED, "batch phase %d cannot be resident", ph);
        const int64_t resident = (int64_t)per_cu * cus;
        const int64_t blocks = units < 4 * resident ? units : 4 * resident;
        hipStream_t sk = s;
        if (ax && branch > 0) {
          sk = ax->s[branch - 1];
          if ((e = hip_check(hipStreamWaitEvent(sk, ax->fork, 0), "fork wait"))) return e;
        }
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds_k, sk, hd, fd, w32);
        if ((e = hip_check(hipGetLastError(), "batch phase launch"))) return e;
        if (ax && branch > 0 && (e = hip_check(hipEventRecord(ax->join[branch - 1], sk), "join event"))) return e;
        if (ax) ++branch;
      }
      for (int b = 1; ax && b < branch; ++b)
        if ((e = hip_check(hipStreamWaitEvent(s, ax->join[b - 1], 0), "join wait"))) return e;
    }
    return IH_OK;
  }
  if ((e = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cf, 256, h->lds), "occupancy"))) return e;
  if (per_cu < 1) return set_error(IH_ERR_UNSUPPORTED, "batch kernel cannot be resident (LDS %d)", h->lds);
  const int64_t resident = (int64_t)per_cu * cus;
  void *args[] = {(void *)&hd, (void *)&fd, (void *)&w32};
  // A cooperative launch recorded by stream capture becomes a plain kernel
  // node, whose grid barrier then has no co-residency guarantee, so the
  // cooperative mode refuses to be captured (the phased mode is the one to
  // capture in a graph).
  hipStreamCaptureStatus ccs = hipStreamCaptureStatusNone;
  if ((e = hip_check(hipStreamIsCapturing(s, &ccs), "hipStreamIsCapturing"))) return e;
  if (ccs != hipStreamCaptureStatusNone)
    return set_error(IH_ERR_UNSUPPORTED,
                     "the cooperative batch launch cannot be captured in a graph (capture the phased mode)");
  return hip_check(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(cf), dim3((unsigned)resident),
                                              dim3(256), args, (unsigned)h->lds, s),
                   "cooperative batch launch");
}
