/*
 * ih_lp.h - C ABI of the learned candidate proposal (libih.so).
 *
 * The thesis scores every candidate window of the search region with the
 * spatial-pyramid distance (Chapter 2, Eqs. 2.23-2.24) and names learned
 * models as a direction it does not build.  This library adds one: a small
 * convolutional network that looks at a crop of the 7 feature channels
 * (R, G, B, intensity, gradient orientation, gradient magnitude, edges; the
 * fused features of the tracker of Sec. 2.4.3-2.4.4) centred on the previous target
 * position and scores each of the 65 x 65 candidate offsets (-32..32 pixels per
 * axis).  The tracker then scores only the k best-ranked offsets exactly.
 *
 * Network, for one crop (all tensors NCHW, batch-major, device memory):
 *   x  [7][128][128]   bf16(feature / 255), 0 outside the frame
 *   a1 [32][64][64]    bf16(relu(conv3x3(x,  W1, stride 2, pad 1) + b1))
 *   a2 [32][64][64]    bf16(relu(conv3x3(a1, W2, dilation 3, pad 3) + b2))
 *   a3 [32][64][64]    bf16(relu(conv3x3(a2, W3, dilation 9, pad 9) + b3))
 *   s  [64][64]        sum_c wh[c] a3[c] + bh
 *   logits[dy][dx]     bilinear(s, 32 + dy/2, 32 + dx/2)      [65][65]
 * Training minimises the softmax cross-entropy of the logits against the
 * offset of the true target, by SGD with momentum.
 *
 * Parameters live in one FP32 array (20,577 floats, the master copy):
 *   W1[32][7][3][3] b1[32] W2[32][32][3][3] b2[32] W3[32][32][3][3] b3[32]
 *   wh[32] bh[1]
 * ih_lp_pack derives the BF16 operands the convolutions read.  bf16 values
 * are passed as uint16_t bit patterns; every rounding to bf16 is
 * round-to-nearest-even.  Convolutions, input gradients and weight gradients
 * run on the BF16 matrix cores with FP32 accumulation; every reduction runs in
 * a fixed order, so results are deterministic.
 *
 * All functions are asynchronous on `stream` (a hipStream_t, NULL = default
 * stream) and return IH_OK or a negative ih_status from ih.h after host-side
 * argument checks; ih_last_error() describes the failure.  No function
 * allocates device memory: the caller owns every buffer.
 */
#ifndef IH_LP_H
#define IH_LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * ih_lp_conv - 3x3 convolution with 32 output channels.
 *   in    [B][Cin][Hin][Win] bf16.
 *   w     [32][9*Cpad] bf16, Cpad = Cin rounded up to a multiple of 8, tap-major:
 *         column k = (kh*3 + kw)*Cpad + ci, zero for ci >= Cin; 8-byte aligned.
 *   out   [B][32][Hout][Wout] bf16, Hout = (Hin + 2 pad - 2 dil - 1)/stride + 1.
 *   mask  NULL: out = bf16(relu(conv + bias)) (forward; bias is [32] FP32).
 *         else [B][32][Hout][Wout] bf16: out = bf16(conv * (mask > 0)), bias
 *         unused (input gradient through a ReLU: pass dZ of the next layer as
 *         `in`, the packed transposed weights as `w`, and that layer's input
 *         activation as `mask`).
 * Cin must not exceed 512.
 */
int ih_lp_conv(const uint16_t *in, int32_t B, int32_t Cin, int32_t Hin,
               int32_t Win, const uint16_t *w, const float *bias,
               int32_t stride, int32_t dil, int32_t pad, const uint16_t *mask,
               uint16_t *out, void *stream);

/*
 * Bytes of FP32 workspace ih_lp_wgrad needs: one 32 x (Cin*9 + 1) partial sum
 * per chunk of `chunk` output pixels (0 for invalid shapes).
 */
size_t ih_lp_wgrad_workspace(int32_t B, int32_t Cin, int32_t Hin, int32_t Win,
                             int32_t stride, int32_t dil, int32_t pad,
                             int64_t chunk);

/*
 * ih_lp_wgrad - weight and bias gradients of a 3x3 convolution.
 *   in  [B][Cin][Hin][Win] bf16 (the layer input), dz [B][32][Hout][Wout] bf16
 *   (gradient of the pre-activation).
 *   dw  out: [32][Cin][3][3] FP32 = sum over batch and pixels of dz * im2col(in)
 *   db  out: [32] FP32 = sum of dz per channel (the product of dz with an
 *       extra column of ones, computed with the weights).
 *   chunk  output pixels per partial sum (positive multiple of 8, at most
 *          65,535 chunks); partials are added in chunk order, so results are
 *          bit-reproducible for a given chunk.
 */
int ih_lp_wgrad(const uint16_t *in, const uint16_t *dz, int32_t B, int32_t Cin,
                int32_t Hin, int32_t Win, int32_t stride, int32_t dil,
                int32_t pad, int64_t chunk, float *ws, size_t ws_bytes,
                float *dw, float *db, void *stream);

/*
 * ih_lp_head - score map and offset logits.
 *   a3 [B][32][64][64] bf16, wh [32], bh [1] FP32; logits out [B][65][65] FP32,
 *   logits[b][dy+32][dx+32] = bilinear(s_b, 32 + dy/2, 32 + dx/2).
 */
int ih_lp_head(const uint16_t *a3, const float *wh, const float *bh, int32_t B,
               float *logits, void *stream);

/*
 * ih_lp_softmax_ce - per-sample loss and logit gradient.
 *   labels [B] in [0, 4225) (index (dy+32)*65 + dx+32 of the true offset).
 *   loss out [B] = -log softmax(logits_b)[label_b];
 *   dlogits out [B][4225] = (softmax - onehot) / B  (gradient of the mean).
 */
int ih_lp_softmax_ce(const float *logits, const int32_t *labels, int32_t B,
                     float *loss, float *dlogits, void *stream);

/*
 * ih_lp_head_bwd - backward of the head and the bilinear sampling.
 *   ds  out [B][64][64] FP32 gradient of the score map.
 *   dz3 out [B][32][64][64] bf16 = bf16(ds * wh[c] * (a3 > 0)).
 *   dwh out [32], dbh out [1] FP32.
 *   ws  FP32 workspace of B * 33 floats (per-sample partial sums, added in
 *       sample order).
 */
int ih_lp_head_bwd(const float *dlogits, const uint16_t *a3, const float *wh,
                   int32_t B, float *ds, uint16_t *dz3, float *dwh, float *dbh,
                   float *ws, void *stream);

/*
 * ih_lp_crop - network inputs from a stack of planar u8 feature frames.
 *   feat [F][C][H][W] u8; frames [B] int32 frame index per crop (NULL: all
 *   from frame 0); centers [B][2] (row, column) int32;
 *   x out [B][C][side][side] bf16 with x[b][c][i][j] =
 *   feat[frames[b]][c][row_b - side/2 + i][col_b - side/2 + j] / 255, and 0
 *   outside the frame or for a frame index outside [0, F).  side must be even.
 */
int ih_lp_crop(const uint8_t *feat, int32_t F, int32_t C, int32_t H, int32_t W,
               const int32_t *frames, const int32_t *centers, int32_t B,
               int32_t side, uint16_t *x, void *stream);

/*
 * ih_lp_origins - candidate window origins from offset indices.
 *   idx   [B][k] int32 offset indices (as from ih_lp_topk), or NULL for all
 *         (2 radius + 1)^2 offsets in index order (then k must equal that).
 *   base  [B][2] int32 window origin of the previous position.
 *   origins out [B][k][2] = base + (o / n - radius, o % n - radius), n = 2 radius + 1;
 *   an index outside [0, n^2) gives an origin far outside every frame, which
 *   ih_match_candidates scores as +inf.
 */
int ih_lp_origins(const int32_t *idx, int32_t B, int32_t k,
                  const int32_t *base, int32_t radius, int32_t *origins,
                  void *stream);

/*
 * ih_lp_pack - BF16 operands from the FP32 parameter array, in the tap-major
 *   layout of ih_lp_conv: w1 [32][72] (Cpad = 8, channel 7 zero), w2, w3
 *   [32][288], and the transposed, tap-flipped w2t, w3t [32][288] used for
 *   input gradients: wt[ci][(kh*3 + kw)*32 + co] = W[co][ci][2-kh][2-kw].
 */
int ih_lp_pack(const float *params, uint16_t *w1, uint16_t *w2, uint16_t *w3,
               uint16_t *w2t, uint16_t *w3t, void *stream);

/*
 * ih_lp_sgd - SGD with momentum and L2 weight decay on n FP32 values:
 *   v <- momentum v + (g + weight_decay p);  p <- p - lr v.
 */
int ih_lp_sgd(float *params, const float *grads, float *mom, int32_t n,
              float lr, float momentum, float weight_decay, void *stream);

/*
 * ih_lp_topk - per sample, the indices of the k largest of n logits
 * (n <= 8192, k <= min(n, 1024)), best first, ties to the lower index, -0
 * equal to +0, NaN below every number.  idx out [B][k] int32.
 */
int ih_lp_topk(const float *logits, int32_t B, int32_t n, int32_t k,
               int32_t *idx, void *stream);

/*
 * Device-resident tracking.  The state of one target lives in device memory,
 * so a sequence of frames is enqueued without host round trips, and the
 * per-frame step can be captured once in a HIP graph and replayed.  Per frame:
 *   ih_track_fetch                   copy frame st->frame of a resident stack
 *                                    into the buffer the build reads
 *   ih_build                         integral histogram of that buffer
 *   ih_track_prepare                 base = previous origin, crop centre
 *   (learned) crop, network, ih_lp_topk, ih_lp_origins, ih_match_candidates
 *   over the k proposals, then ih_track_gate, or (bounded) the pyramid
 *   distances of all offsets with one level fewer and ih_track_gate_bounded
 *   (exhaustive only) ih_lp_origins over all offsets
 *   ih_match_candidates over the exhaustive list, ih_track_commit
 * The gate implements the fallback rule: the best proposal is accepted when
 * its distance d satisfies d <= (1 + tau) * dist (evaluated in double);
 * then the exhaustive list is filled with origins outside every frame, so the
 * exhaustive scoring returns best = -1 without reading the histogram.  The
 * bounded gate keeps instead the offsets that could still beat d, so the
 * result is always the exhaustive search's.
 */
typedef struct {
  int32_t origin[2]; /* window origin (row, column) accepted at the previous frame */
  float dist;        /* its distance d*                                           */
  int32_t decision;  /* accepted offset index, -1 (full exhaustive list) or -2    */
                     /* (bounded list), written by prepare and the gates          */
  int32_t frame;     /* frame being processed; ih_track_commit advances it        */
  int32_t scored;    /* candidates the exhaustive list holds this frame (written   */
                     /* by prepare and the gates)                                  */
} ih_track_state;

/* dst [frame_bytes] = stack [st->frame * frame_bytes ...]; nothing is copied
   when st->frame is outside [0, n_frames).  stack, dst and frame_bytes must be
   multiples of 16 bytes. */
int ih_track_fetch(const void *stack, int64_t frame_bytes, int32_t n_frames,
                   const ih_track_state *st, void *dst, void *stream);

/* base [2] = st->origin; center [2] (may be NULL) = origin + (win_h/2, win_w/2);
   st->decision = -1, st->scored = 0. */
int ih_track_prepare(ih_track_state *st, int32_t win_h, int32_t win_w,
                     int32_t *base, int32_t *center, void *stream);

/* Reads the k-proposal search (idx [k] offset indices, kdist [k], kbest [1]
   from ih_match_candidates); sets st->decision and st->scored (0 when the
   proposal is accepted, (2 radius + 1)^2 otherwise) and writes exh_origins
   [(2 radius + 1)^2][2]. */
int ih_track_gate(ih_track_state *st, const int32_t *idx, const float *kdist,
                  const int32_t *kbest, int32_t radius, double tau,
                  const int32_t *base, int32_t *exh_origins, void *stream);

/* Bounded form of ih_track_gate, which keeps the search exact.  When the
   margin rule accepts the best proposal (distance d <= (1 + tau) * dist), the
   exhaustive list keeps only the offsets whose lower bound lb [(2 radius +
   1)^2] does not exceed d, within a relative 2^-16 for rounding; the others
   get origins outside every frame.  lb is the pyramid distance of each
   offset with one level fewer (ih_match_candidates with levels - 1 levels
   over all offsets and the leading part of the template descriptor, metric
   chi2 or L1): merging cells never raises a chi-square or L1 sum, so the
   level sums grow with the level, and the Eq. 2.24 distance of L + 1 levels
   minus that of L levels is a non-negative combination of those sums'
   differences; so the scoring of that list returns the exhaustive search's
   argmin and distance (ties included).  Otherwise (a fallback) every offset is
   listed.  st->decision = -2 (bounded) or -1 (fallback); st->scored = the
   number of listed offsets. */
int ih_track_gate_bounded(ih_track_state *st, const float *kdist,
                          const int32_t *kbest, int32_t radius, double tau,
                          const int32_t *base, const float *lb,
                          int32_t *exh_origins, void *stream);

/* New state from the accepted proposal (kdist, kbest; st->decision >= 0) or
   the exhaustive list's search (exh_dist, exh_best; +inf and the old origin
   when no candidate was inside).  Record f = st->frame of rec [n_rec][5]
   (when f < n_rec) receives origin row, origin column, the distance's FP32
   bits, 1 when the gate fell back to the full exhaustive list (0 otherwise),
   and st->scored; then st->frame = f + 1. */
int ih_track_commit(ih_track_state *st, const float *kdist,
                    const int32_t *kbest, const float *exh_dist,
                    const int32_t *exh_best, int32_t radius, int32_t *rec,
                    int32_t n_rec, void *stream);

/* Search region of the frame (C x H x W uint8): the (2 radius + win_h) x
   (2 radius + win_w) block around st->origin that holds every candidate
   window of the offsets -radius..radius, shifted inside the frame (it must
   fit: IH_ERR_RANGE otherwise), is copied to region [C][rh][rw], and
   rbase [2] receives st->origin in region coordinates.  The candidate search
   over the region's integral histogram with origins rbase + offset gives the
   same distances as over the frame's (windows inside the frame lie inside the
   region; windows leaving the frame leave the region), so a tracker need not
   build the frame's whole histogram. */
int ih_track_region(const void *frame, int32_t C, int32_t H, int32_t W,
                    const ih_track_state *st, int32_t radius, int32_t win_h,
                    int32_t win_w, void *region, int32_t *rbase, void *stream);

/* Local refinement of the best proposal.  refine_origins writes the origins
   base + offset of the (2q+1)^2 offsets around idx[kbest[0]] (row-major; an
   offset outside -radius..radius gets an origin outside every frame; all of
   them when kbest[0] < 0).  After ih_match_candidates over those origins
   (ndist, nbest), refine_pick keeps the better of the current best and the
   neighbourhood's best (smaller distance, or equal distance at a lower offset
   index, the exhaustive search's tie rule) and stores it in slot 0:
   idx[0] = offset index, kdist[0] = distance, kbest[0] = 0.  1 <= q <= 32. */
int ih_track_refine_origins(const int32_t *idx, const int32_t *kbest, int32_t q,
                            int32_t radius, const int32_t *base,
                            int32_t *origins, void *stream);
int ih_track_refine_pick(int32_t *idx, float *kdist, int32_t *kbest,
                         const float *ndist, const int32_t *nbest, int32_t q,
                         int32_t radius, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IH_LP_H */
