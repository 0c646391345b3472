"""Pyramid-histogram tracking with exhaustive and learned candidate search.

Per frame the integral histogram of the feature channels is built (Chapter 2);
candidate windows around the previous target position are scored by their
spatial-pyramid distance to the frame-0 template (Eqs. 2.23-2.24) and the best
one becomes the new position, the sliding-window search of the thesis's
tracker.  Two searches:

* exhaustive: all 65 x 65 window offsets (-32..32 px per axis);
* learned: the proposal network ranks the offsets from a crop centred on the
  previous position, only the top k are scored exactly, the best of them is
  optionally moved by a local search among its neighbouring offsets, and
  the exhaustive search runs instead whenever the result scores worse than
  the margin (1 + tau) d*, where d* is the distance accepted at the previous
  frame.  In the bounded form an accepted result d only narrows the
  exhaustive search: the pyramid distance of every offset with one level
  fewer is a lower bound of its full pyramid distance, and only the offsets
  whose bound does not exceed d are scored exactly, which returns the
  exhaustive search's own result.

Either search can run on the integral histogram of the whole frame (as the
thesis's tracker does) or of the search region only.  All scoring, network
and index work runs in libih.so with the target state on the device; the
host reads the records back once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import proposal as lp
from .ih import (IHError, TileCfg, _check, _p, _stream, ih_build, ih_match_candidates, ih_pyramid_desc, lib,
                 shape_of, workspace_size)

RADIUS = lp.RADIUS
N_OFF = lp.N_OFFSETS


class PyramidTracker:
    """Exhaustive pyramid-distance search over one frame size.

    With ``region`` the tracker never builds a whole frame's integral
    histogram: per frame it copies the search region around the previous
    origin (every candidate window of the 65 x 65 offsets, shifted inside the
    frame) and builds that region's histogram; candidate origins are then
    given in region coordinates.  Distances and the chosen window are the
    same as with the frame's histogram."""

    def __init__(self, H: int, W: int, C: int = 7, bins: int = 16, levels: int = 3, metric: str = "chi2",
                 layout: str = "hwb", cfg: Optional[TileCfg] = None, device="cuda", region: bool = False):
        self.H, self.W, self.C, self.bins, self.levels = H, W, C, bins, levels
        self.metric, self.layout, self.cfg, self.region = metric, layout, cfg, region
        self.P = C * bins
        dev = torch.device(device)
        self.device = dev
        self.ih = None
        self.ws = None
        if not region:
            self._alloc(H, W)
        self.origins = torch.empty((N_OFF, 2), dtype=torch.int32, device=dev)
        self.dist = torch.empty(N_OFF, dtype=torch.float32, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)
        self.base = torch.empty((1, 2), dtype=torch.int32, device=dev)   # previous origin (frame coordinates)
        self.sbase = self.base if not region else torch.empty((1, 2), dtype=torch.int32, device=dev)
        self.tmpl = None
        self.win = None

    def _alloc(self, h, w):
        self.ih = torch.empty(shape_of(self.P, h, w, self.layout), dtype=torch.int32, device=self.device)
        self.ws = torch.empty(max(1, workspace_size(h, w, self.C, self.bins, False, self.cfg, self.layout)),
                              dtype=torch.uint8, device=self.device)

    def build(self, feat: torch.Tensor):
        """Integral histogram of a whole frame (frame mode)."""
        ih_build(feat, self.bins, out=self.ih, ws=self.ws, cfg=self.cfg, layout=self.layout)

    def set_template(self, feat0: torch.Tensor, box: Sequence[int]):
        """Template = pyramid descriptor of window box = (row, col, h, w) in feat0."""
        wins = torch.tensor([list(box)], dtype=torch.int32, device=self.device)
        if self.region:
            full = ih_build(feat0, self.bins, cfg=None, layout=self.layout)
            self.tmpl = ih_pyramid_desc(full, wins, self.levels, layout=self.layout).reshape(-1).clone()
            del full
            h, w = int(box[2]), int(box[3])
            if self.win != (h, w):
                self.rh, self.rw = 2 * RADIUS + h, 2 * RADIUS + w
                self.reg = torch.empty((self.C, self.rh, self.rw), dtype=torch.uint8, device=self.device)
                self._alloc(self.rh, self.rw)
        else:
            self.build(feat0)
            self.tmpl = ih_pyramid_desc(self.ih, wins, self.levels, layout=self.layout).reshape(-1).clone()
        self.win = (int(box[2]), int(box[3]))

    def frame_step(self, cur: torch.Tensor, state: torch.Tensor):
        """Enqueue this frame's histogram: of the whole frame, or of the search
        region around state's origin (which also sets sbase)."""
        if not self.region:
            self.build(cur)
            return
        h, w = self.win
        _check(lib().ih_track_region(_p(cur), self.C, self.H, self.W, _p(state), RADIUS, h, w, _p(self.reg),
                                     _p(self.sbase), _stream(cur)), "ih_track_region")
        ih_build(self.reg, self.bins, out=self.ih, ws=self.ws, cfg=self.cfg, layout=self.layout)

    def score(self, origins: torch.Tensor, dist: torch.Tensor, best: torch.Tensor):
        return ih_match_candidates(self.ih, self.tmpl, self.win[0], self.win[1], origins, self.levels,
                                   self.metric, dist, best, self.layout)

    def score_coarse(self, origins: torch.Tensor, dist: torch.Tensor, best: torch.Tensor):
        """Pyramid distances with one level fewer (the template's descriptor
        of those levels is the leading part of its full descriptor): a lower
        bound of each candidate's pyramid distance."""
        lv = max(1, self.levels - 1)
        n = self.P * sum(4 ** l for l in range(lv))
        return ih_match_candidates(self.ih, self.tmpl[:n], self.win[0], self.win[1], origins, lv,
                                   self.metric, dist, best, self.layout)


class LearnedTracker:
    """Top-k proposals from the network, exact scoring, optional local
    refinement of the best proposal, exhaustive fallback."""

    def __init__(self, tracker: PyramidTracker, net: Optional[lp.ProposalNet], k: int = 64, tau: float = 0.25,
                 prior_logits: Optional[torch.Tensor] = None, refine_rounds: int = 0, refine_q: int = 2,
                 bound: bool = False):
        """net=None with prior_logits ranks the offsets by a fixed score instead
        of the network (the no-network baseline).  refine_rounds rounds of the
        local search move the best candidate to the best of the (2 refine_q + 1)^2
        offsets around it.  With bound, an accepted result narrows the
        exhaustive search by a lower bound (the pyramid distance with one level
        fewer) instead of replacing it
        (the track then always equals the exhaustive one)."""
        if net is None and prior_logits is None:
            raise IHError("need a network or fixed prior logits")
        if tracker.metric == "pmk":
            raise IHError("the fallback rule needs a distance (chi2 or l1); pmk is a similarity")
        self.tr, self.net, self.k, self.tau = tracker, net, k, tau
        self.rounds, self.q = int(refine_rounds), int(refine_q)
        self.bound = bool(bound)
        dev = tracker.device
        if self.bound:
            self.allorig = torch.empty((N_OFF, 2), dtype=torch.int32, device=dev)
            self.lb = torch.empty(N_OFF, dtype=torch.float32, device=dev)
            self.lbbest = torch.empty(1, dtype=torch.int32, device=dev)
        self.prior = prior_logits
        self.idx = torch.empty((1, k), dtype=torch.int32, device=dev)
        self.korig = torch.empty((k, 2), dtype=torch.int32, device=dev)
        self.kdist = torch.empty(k, dtype=torch.float32, device=dev)
        self.kbest = torch.empty(1, dtype=torch.int32, device=dev)
        self.center = torch.empty((1, 2), dtype=torch.int32, device=dev)
        m = 2 * self.q + 1
        self.norig = torch.empty((m * m, 2), dtype=torch.int32, device=dev)
        self.ndist = torch.empty(m * m, dtype=torch.float32, device=dev)
        self.nbest = torch.empty(1, dtype=torch.int32, device=dev)

    def propose(self, feat: torch.Tensor, origin=None):
        """Enqueue the ranking of the offsets; fills self.idx.  The crop is
        centred on the window at origin, or at self.center as already set on
        the device when origin is None."""
        if self.net is None:
            lp.lp_topk(self.prior.view(1, -1), self.k, self.idx)
            return
        if origin is not None:
            h, w = self.tr.win
            self.center.copy_(torch.tensor([[int(origin[0]) + h // 2, int(origin[1]) + w // 2]],
                                           dtype=torch.int32))
        x = self.net.crop(feat, self.center)
        logits = self.net.forward(x)
        lp.lp_topk(logits.view(1, -1), self.k, self.idx)

    def search(self, cur: torch.Tensor):
        """Enqueue proposals, their exact scores and the local refinement."""
        tr, L = self.tr, lib()
        self.propose(cur)
        lp.lp_origins(tr.sbase, RADIUS, idx=self.idx, out=self.korig)
        tr.score(self.korig, self.kdist, self.kbest)
        s = _stream(cur)
        for _ in range(self.rounds):
            _check(L.ih_track_refine_origins(_p(self.idx), _p(self.kbest), self.q, RADIUS, _p(tr.sbase),
                                             _p(self.norig), s), "ih_track_refine_origins")
            tr.score(self.norig, self.ndist, self.nbest)
            _check(L.ih_track_refine_pick(_p(self.idx), _p(self.kdist), _p(self.kbest), _p(self.ndist),
                                          _p(self.nbest), self.q, RADIUS, s), "ih_track_refine_pick")
        if self.bound:
            lp.lp_origins(tr.sbase, RADIUS, out=self.allorig)
            tr.score_coarse(self.allorig, self.lb, self.lbbest)

    def gate(self, state: torch.Tensor, exh: torch.Tensor):
        """Enqueue the fallback rule (plain or bounded), filling exh."""
        tr, L = self.tr, lib()
        s = _stream(state)
        if self.bound:
            _check(L.ih_track_gate_bounded(_p(state), _p(self.kdist), _p(self.kbest), RADIUS, float(self.tau),
                                           _p(tr.sbase), _p(self.lb), _p(exh), s), "ih_track_gate_bounded")
        else:
            _check(L.ih_track_gate(_p(state), _p(self.idx), _p(self.kdist), _p(self.kbest), RADIUS,
                                   float(self.tau), _p(tr.sbase), _p(exh), s), "ih_track_gate")


@dataclass
class Track:
    origins: np.ndarray       # T x 2 window origins
    dists: np.ndarray         # T accepted distances
    fallback: np.ndarray      # T bool (learned search only)
    scored: Optional[np.ndarray] = None  # T, candidates of the exhaustive list scored exactly


class _Stepper:
    """One frame's step with the target state on the device: fetch the frame
    into a fixed buffer, build (frame or search region), search (learned with
    its fallback rule, or exhaustive), commit the new state and its record."""

    def __init__(self, frames: torch.Tensor, box0, tracker: PyramidTracker, learned: Optional[LearnedTracker]):
        if frames.dim() != 4 or frames.dtype != torch.uint8 or not frames.is_contiguous():
            raise IHError("frames must be a contiguous T x C x H x W uint8 tensor")
        if tracker.metric == "pmk":
            raise IHError("the tracker minimises a distance (chi2 or l1); pmk is a similarity")
        self.frames, self.tr, self.learned = frames, tracker, learned
        self.T = frames.shape[0]
        dev = tracker.device
        tracker.set_template(frames[0], box0)
        # ih_track_state: origin, dist 0.0, decision, frame 1, scored
        self.state = torch.from_numpy(np.array([box0[0], box0[1], 0, -1, 1, 0], np.int32)).to(dev)
        self.exh = torch.empty((N_OFF, 2), dtype=torch.int32, device=dev)
        self.rec = torch.zeros((self.T, 5), dtype=torch.int32, device=dev)
        self.rec[0, 0], self.rec[0, 1] = int(box0[0]), int(box0[1])
        self.cur = torch.empty(frames.shape[1:], dtype=torch.uint8, device=dev)
        self.use_net = learned is not None and learned.net is not None
        if self.use_net and not learned.net.packed:
            learned.net.pack()

    def set_state(self, t: int, origin, dist: float):
        st = np.array([int(origin[0]), int(origin[1]), 0, -1, t, 0], np.int32)
        st[2] = np.array([dist], np.float32).view(np.int32)[0]
        self.state.copy_(torch.from_numpy(st))

    def step(self):
        L, tr, lt = lib(), self.tr, self.learned
        s = _stream(self.state)
        h, w = tr.win
        _check(L.ih_track_fetch(_p(self.frames), self.cur.numel(), self.T, _p(self.state), _p(self.cur), s),
               "ih_track_fetch")
        _check(L.ih_track_prepare(_p(self.state), h, w, _p(tr.base), _p(lt.center) if self.use_net else None, s),
               "ih_track_prepare")
        tr.frame_step(self.cur, self.state)
        if lt is not None:
            lt.search(self.cur)
            lt.gate(self.state, self.exh)
        else:
            lp.lp_origins(tr.sbase, RADIUS, out=self.exh)
        tr.score(self.exh, tr.dist, tr.best)
        _check(L.ih_track_commit(_p(self.state), _p(lt.kdist) if lt is not None else None,
                                 _p(lt.kbest) if lt is not None else None, _p(tr.dist), _p(tr.best), RADIUS,
                                 _p(self.rec), self.T, s), "ih_track_commit")

    def result(self) -> Track:
        r = self.rec.cpu().numpy()
        fb = r[:, 3].astype(bool) if self.learned is not None else np.zeros(self.T, bool)
        return Track(r[:, :2].astype(np.int64), r[:, 2].copy().view(np.float32).astype(np.float64), fb,
                     r[:, 4].astype(np.int64))


def track(frames: torch.Tensor, box0, tracker: PyramidTracker, learned: Optional[LearnedTracker] = None,
          teacher: Optional[Track] = None) -> Track:
    """Track through a resident T x C x H x W uint8 stack, one frame at a time.
    With `teacher`, every search starts from the teacher's previous position
    and distance (per-frame agreement)."""
    st = _Stepper(frames, box0, tracker, learned)
    for t in range(1, st.T):
        if teacher is not None:
            st.set_state(t, teacher.origins[t - 1], float(teacher.dists[t - 1]))
        st.step()
    return st.result()


def track_device(frames: torch.Tensor, box0, tracker: PyramidTracker, learned: Optional[LearnedTracker] = None,
                 graph: bool = False) -> Track:
    """The free-running track() with every step enqueued without a host round
    trip; with `graph`, the step is captured once in a HIP graph and replayed
    per frame.  Returns the same track as track(frames, box0, tracker, learned)."""
    st = _Stepper(frames, box0, tracker, learned)
    if graph and st.T > 1:
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            st.step()
        for _ in range(1, st.T):
            g.replay()
    else:
        for _ in range(1, st.T):
            st.step()
    return st.result()


def distance_prior() -> torch.Tensor:
    """Fixed ranking of the offsets by distance from the previous position
    (-(dy^2 + dx^2)): the search without a network."""
    d = np.arange(-RADIUS, RADIUS + 1)
    return torch.tensor(-(d[:, None] ** 2 + d[None, :] ** 2).astype(np.float32).reshape(1, -1))


# ---------------------------------------------------------------- training --
@dataclass
class Samples:
    frame: np.ndarray          # n, index into the frame stack
    center: np.ndarray         # n x 2, crop centre of the previous window
    offset: np.ndarray         # n x 2, displacement chosen by the exhaustive search


def samples_from_track(trk: Track, win, frame0: int = 0) -> Samples:
    """Frame t of a track gives one sample: crop of frame t centred on the
    window at t-1, labelled with the exhaustive search's displacement."""
    h, w = win
    prev = trk.origins[:-1]
    off = trk.origins[1:] - prev
    ok = np.all(np.abs(off) <= RADIUS, axis=1) & np.isfinite(trk.dists[1:])
    t = np.arange(1, len(trk.origins))[ok]
    center = prev[ok] + np.array([h // 2, w // 2])
    return Samples(frame0 + t, center, off[ok])


def concat(samples: List[Samples]) -> Samples:
    return Samples(np.concatenate([s.frame for s in samples]), np.concatenate([s.center for s in samples]),
                   np.concatenate([s.offset for s in samples]))


def train(net: lp.ProposalNet, stack: torch.Tensor, samples: Samples, steps: int, batch: int = 64,
          lr: float = 0.02, momentum: float = 0.9, weight_decay: float = 1e-4, jitter: int = 12,
          seed: int = 0, log_every: int = 0, cosine: bool = True) -> List[float]:
    """SGD on random batches of samples.  Each draw shifts the crop centre by a
    random jitter j (|j| <= jitter per axis) and the label by -j, so the
    network sees the target at many positions; labels stay inside the
    search range.  With `cosine` the learning rate decays as
    lr (1 + cos(pi s / steps)) / 2.  Returns the mean loss of every step
    (read back every `log_every` steps, or at the end)."""
    rng = np.random.default_rng(seed)
    dev = net.device
    n = len(samples.frame)
    losses = []
    pending = []
    fr_d = torch.empty(batch, dtype=torch.int32, device=dev)
    ce_d = torch.empty((batch, 2), dtype=torch.int32, device=dev)
    lb_d = torch.empty(batch, dtype=torch.int32, device=dev)
    for s in range(steps):
        pick = rng.integers(0, n, batch)
        j = rng.integers(-jitter, jitter + 1, (batch, 2))
        off = samples.offset[pick]
        j = np.clip(j, off - RADIUS, off + RADIUS)
        lab = lp.label_of(off[:, 0] - j[:, 0], off[:, 1] - j[:, 1])
        fr_d.copy_(torch.from_numpy(samples.frame[pick].astype(np.int32)))
        ce_d.copy_(torch.from_numpy((samples.center[pick] + j).astype(np.int32)))
        lb_d.copy_(torch.from_numpy(lab.astype(np.int32)))
        x = net.crop(stack, ce_d, frames=fr_d)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps)) if cosine else lr
        loss = net.train_step(x, lb_d, lr_s, momentum, weight_decay)
        pending.append(loss.mean())
        if (log_every and (s + 1) % log_every == 0) or s == steps - 1:
            losses.extend(float(v) for v in torch.stack(pending).cpu())
            pending = []
            if log_every:
                print("step %d loss %.4f" % (s + 1, losses[-1]), flush=True)
    return losses


def recall(net_or_prior, stack: torch.Tensor, samples: Samples, k: int = 64, batch: int = 64) -> float:
    """Fraction of samples whose exhaustive displacement is among the top k."""
    hits = 0
    n = len(samples.frame)
    for s in range(0, n, batch):
        e = min(n, s + batch)
        if isinstance(net_or_prior, lp.ProposalNet):
            net = net_or_prior
            x = net.crop(stack, torch.from_numpy(samples.center[s:e].astype(np.int32)).to(net.device),
                         frames=torch.from_numpy(samples.frame[s:e].astype(np.int32)).to(net.device))
            idx = lp.lp_topk(net.forward(x).view(e - s, -1), k).cpu().numpy()
        else:
            prior = net_or_prior.view(1, -1)
            idx = np.repeat(lp.lp_topk(prior, k).cpu().numpy(), e - s, 0)
        lab = lp.label_of(samples.offset[s:e, 0], samples.offset[s:e, 1])
        hits += int(np.sum(np.any(idx == lab[:, None], axis=1)))
    return hits / max(1, n)
