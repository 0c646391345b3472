/*
 * ih.h - C ABI of the MI355X (gfx950) integral-histogram library, libih.so.
 *
 * The library computes the integral histogram of binned image channels and
 * the constant-time region descriptors built on it, after Poostchi 2017
 * (arXiv:1711.01656): the integral histogram (Eq. 2.15, Alg. 5), four-corner
 * region histograms (Eq. 2.16), spatially weighted local histograms (SWIH,
 * Eq. 3.1, 3.3, 3.4, Sec. 3.1.3), spatial-pyramid descriptors (Alg. 2,
 * Sec. 2.4.4) and exhaustive pyramid-distance candidate search (Sec. 2.4.3,
 * Eq. 2.22-2.24).
 *
 * General conventions
 *   - Every pointer argument named as "device" is GPU memory owned by the
 *     caller; the library never allocates, never frees and keeps no pointer
 *     after the call returns.  Scratch memory is a caller-supplied workspace.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  Argument errors are detected on the host before anything is
 *     enqueued; the call then returns a negative IH_ERR_* code, enqueues
 *     nothing, and ih_last_error() describes the problem.  No call aborts or
 *     throws.  Problems that only the device can see (an out-of-frame
 *     rectangle) are reported in-band with the sentinels documented per call.
 *   - Images are C planar channels of H x W unsigned 8- or 16-bit values.
 *     A value v of a `value_bits`-bit channel falls into bin
 *     floor(v * bins / 2^value_bits) (equal-width bins; the thesis leaves the
 *     edges open, Eq. 2.15's Q).  Plane p = channel * bins + bin; P = C * bins.
 *   - Integral histograms hold P x H x W int32 values, inclusive: H(p, r, c)
 *     counts pixels of plane p in rows 0..r and columns 0..c (Eq. 2.15).
 *     Rows are the thesis's x, columns its y.  They are stored bin-major
 *     (IH_BHW, the thesis's layout, Sec. 5.1.1, Fig. 5.1) or planes-innermost
 *     (IH_HWB); see ih_layout.
 *   - Rectangles are half-open {r0, c0, r1, c1}: rows r0..r1-1, columns
 *     c0..c1-1.
 */
#ifndef IH_H
#define IH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IH_OK 0
#define IH_ERR_INVALID_ARG (-1) /* a size, pointer or enum is invalid       */
#define IH_ERR_RANGE (-2)       /* a size exceeds what the format can hold   */
#define IH_ERR_OVERFLOW (-3)    /* counts would not fit their integer type   */
#define IH_ERR_UNSUPPORTED (-4) /* valid but not implemented combination     */
#define IH_ERR_HIP (-5)         /* the HIP runtime reported an error         */
#define IH_ERR_WORKSPACE (-6)   /* workspace missing or smaller than needed  */

typedef enum { IH_U8 = 0, IH_U16 = 1 } ih_dtype;
typedef enum { IH_CHI2 = 0, IH_L1 = 1, IH_PMK = 2 } ih_metric;
typedef enum { IH_MANHATTAN = 0, IH_QUADRATIC = 1, IH_GAUSSIAN = 2 } ih_kernel;

/*
 * Memory layout of integral-histogram tensors (and their moment tensors).
 *   IH_BHW  P x H x W, bin-major (Sec. 5.1.1, Fig. 5.1): element (p, r, c) at
 *           (p * H + r) * W + c.  Each plane is contiguous.
 *   IH_HWB  H x W x P, planes innermost: element (p, r, c) at
 *           (r * W + c) * P + p.  The P-bin histogram at one pixel is
 *           contiguous, so a four-corner query reads 4 runs of P values
 *           instead of 4 P scattered values (for query-heavy workloads).
 */
typedef enum { IH_BHW = 0, IH_HWB = 1 } ih_layout;

/* Half-open rectangle: rows [r0, r1), columns [c0, c1). */
typedef struct {
  int32_t r0, c0, r1, c1;
} ih_rect;

/*
 * How the build is organised (ih_tile_cfg.passes).
 *   IH_PASSES_DEFAULT  the library's choice for the shape and layout.
 *   IH_PASSES_ONE      one launch (bin-major layout only): row bands of
 *                      tile_h rows, each swept from left to right in tiles of
 *                      tile_w columns by one wavefront per group of
 *                      planes_per_wave planes, first counting (publishing
 *                      every tile's band aggregate), then writing out with
 *                      its band's row carries on chip; the top boundary of
 *                      every tile comes from the bands above by a look-back
 *                      to the nearest published inclusive bottom row through
 *                      the aggregates in between.  tile_h in [1, 1024];
 *                      tile_w 64, 128 or 256; planes_per_wave 1, 2 or 4.
 *   IH_PASSES_THREE    three passes: per-tile histograms, scans of the tile
 *                      carries, write-out (the shapes below).
 */
#define IH_PASSES_DEFAULT 0
#define IH_PASSES_ONE 1
#define IH_PASSES_THREE 3

/*
 * Tile shape of the build: tiles of tile_h rows by tile_w columns.  With
 * three passes:
 *   IH_BHW: each wavefront of the write-out pass owns one tile and
 *           planes_per_wave consecutive planes of one channel; its lanes map
 *           to columns.  tile_h in [1, 256]; tile_w 64, 128 or 256;
 *           planes_per_wave 1, 2, 4, 8 or 16.
 *   IH_HWB: each wavefront owns one tile and 64 consecutive planes; its lanes
 *           map to planes.  tile_h in [1, 256]; tile_w 16, 32 or 64;
 *           planes_per_wave must be 64.
 * With one pass, see IH_PASSES_ONE.  NULL (or tile_h == 0 with one pass)
 * selects a shape from a built-in heuristic.
 */
typedef struct {
  int32_t tile_h;
  int32_t tile_w;
  int32_t planes_per_wave;
  int32_t passes;           /* IH_PASSES_*                                  */
} ih_tile_cfg;

/*
 * Device status bits of a build, left in the first 4 bytes of its workspace
 * (a uint32) once the build has run; the caller reads them after the stream
 * has reached the end of the build.  Every build clears them first.
 *   IH_STATUS_VALUE_RANGE   some pixel value was >= 2^value_bits (the
 *                           results are then unspecified but the build
 *                           stays in bounds).
 *   IH_STATUS_WAIT_TIMEOUT  a single-pass build's wait for another band gave
 *                           up (after about a second); the build completed
 *                           but its result is invalid.
 */
#define IH_STATUS_VALUE_RANGE 1u
#define IH_STATUS_WAIT_TIMEOUT 2u

/* Library version (major * 10000 + minor * 100 + patch). */
int ih_version(void);

/* Thread-local description of the last error returned on this thread. */
const char *ih_last_error(void);

/*
 * Bytes of workspace ih_build needs for this shape (0 on invalid arguments).
 * moments: non-zero when the coordinate-moment tensors will be requested.
 */
size_t ih_build_workspace_size(int32_t H, int32_t W, int32_t C, int32_t bins,
                               int32_t moments, int32_t layout,
                               const ih_tile_cfg *cfg);

/*
 * ih_build - integral histogram of a binned image (Eq. 2.15; computed by the
 * recurrence of Alg. 5 reorganised into tiles; Sec. 5.1 describes the
 * thesis's own GPU variants).
 *
 *   img         device, C x H x W values of type dtype (IH_U8 or IH_U16).
 *   H, W, C     image rows, columns, channels; H, W, C >= 1 and
 *               H * W < 2^31.
 *   bins        bins per channel, 1..256 and at most 2^value_bits.
 *   value_bits  significant bits per value: 1..8 for IH_U8, 1..16 for
 *               IH_U16.  Every value must be < 2^value_bits; larger values
 *               give unspecified (but in-bounds) results and set
 *               IH_STATUS_VALUE_RANGE in the workspace's status word.
 *   layout      IH_BHW or IH_HWB, for ih and the moment tensors.
 *   ih          device, out: P x H x W int32 integral histogram (in layout).
 *   mom_x,      device, out, both NULL or both non-NULL: P x H x W uint32
 *   mom_y       coordinate-moment integral histograms (in layout)
 *                 Mx(p,r,c) = sum over the same region of row    * [bin = p]
 *                 My(p,r,c) = sum over the same region of column * [bin = p]
 *               stored modulo 2^32.  These are the weighted integral
 *               histograms of Eq. 3.4: every weight affine in the pixel
 *               coordinates is a combination of 1, row and column.  Region
 *               sums taken from them (four corners, modulo 2^32) are exact
 *               whenever the true regional sum is below 2^32.
 *   cfg         tile shape and number of passes, or NULL for the
 *               library's choice.
 *   ws          device workspace of ws_bytes >= ih_build_workspace_size().
 *               Its contents on entry do not matter; after the build its
 *               first word holds the IH_STATUS_* bits, the rest is garbage.
 *               Two builds must not use one workspace at the same time.
 *   stream      hipStream_t.
 * Returns IH_OK or IH_ERR_*.  Outputs must not overlap the image or ws.
 */
int ih_build(const void *img, int32_t dtype, int32_t H, int32_t W, int32_t C,
             int32_t bins, int32_t value_bits, int32_t layout, int32_t *ih,
             uint32_t *mom_x, uint32_t *mom_y, const ih_tile_cfg *cfg,
             void *ws, size_t ws_bytes, void *stream);

/*
 * Bytes of device scratch that ih_build_noalloc has on each GPU (64 MiB).
 */
#define IH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * ih_build_noalloc - ih_build for callers that cannot allocate memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same computation, arguments and results as ih_build, without
 * the workspace: the build uses a scratch array the library holds on each
 * GPU (IH_NOALLOC_SCRATCH_BYTES, set up on the first call on that device and
 * kept until the process ends).  The call allocates nothing and frees
 * nothing.
 *
 *   img ... cfg as for ih_build; the stream must belong to the current
 *               device.
 *   status      device, out, or NULL: receives the build's IH_STATUS_* word
 *               (a uint32) once the stream reaches the end of the build.
 * Returns IH_ERR_WORKSPACE, enqueuing nothing, when the shape needs more than
 * IH_NOALLOC_SCRATCH_BYTES of workspace (ih_build_workspace_size() tells the
 * need); otherwise as ih_build.  Every call on one GPU shares that GPU's
 * scratch array: two calls whose builds overlap in time on one GPU (on
 * different streams, or from different threads) race and both results are
 * undefined; calls ordered on one stream are safe.  Everything the build
 * needs zeroed it clears itself, so stale scratch contents do not matter.
 */
int ih_build_noalloc(const void *img, int32_t dtype, int32_t H, int32_t W,
                     int32_t C, int32_t bins, int32_t value_bits,
                     int32_t layout, int32_t *ih, uint32_t *mom_x,
                     uint32_t *mom_y, const ih_tile_cfg *cfg, uint32_t *status,
                     void *stream);

/*
 * ih_build_weighted - weighted integral histogram: the plane-p entry sums a
 * per-pixel weight instead of counting (Alg. 2 step 4, the PHoG building
 * block: gradient orientation binned, gradient magnitude as the weight, edge
 * pixels only):
 *   G(p,r,c) = sum over r' <= r, c' <= c of
 *              wt(ch,r',c') * [mask(ch,r',c') != 0] * [bin(ch,r',c') = p]
 * with ch = p / bins.  Same tiles, passes and layouts as ih_build.
 *
 *   img, dtype, H, W, C, bins, value_bits, layout, cfg, ws, ws_bytes,
 *   stream      as for ih_build (the workspace size is that of ih_build
 *               without moments: ih_build_workspace_size(..., 0, ...)).
 *   weight      device, C x H x W uint8 weights (not NULL).
 *   mask        device, C x H x W uint8, or NULL: a pixel whose mask byte is
 *               0 contributes nothing; NULL means every pixel contributes.
 *   ih          device, out: P x H x W int32 (in layout).
 * Needs H * W * 255 <= 2^31 - 1 (IH_ERR_OVERFLOW otherwise), so no sum can
 * overflow.  Returns IH_OK or IH_ERR_*.  Outputs must not overlap the inputs
 * or ws.
 */
int ih_build_weighted(const void *img, int32_t dtype, const uint8_t *weight,
                      const uint8_t *mask, int32_t H, int32_t W, int32_t C,
                      int32_t bins, int32_t value_bits, int32_t layout,
                      int32_t *ih, const ih_tile_cfg *cfg, void *ws,
                      size_t ws_bytes, void *stream);

/*
 * ih_query_rect - region histograms by four corner lookups (Eq. 2.16):
 *   h(R, p) = H(r1-1, c1-1) - H(r0-1, c1-1) - H(r1-1, c0-1) + H(r0-1, c0-1)
 * with H(-1, .) = H(., -1) = 0.
 *   ih      device, P x H x W int32 from ih_build, in `layout`.
 *   rects   device, n half-open rectangles.
 *   out     device, out: n x P int32.  An empty rectangle (r0 == r1 or
 *           c0 == c1) gives zeros; a rectangle not satisfying
 *           0 <= r0 <= r1 <= H and 0 <= c0 <= c1 <= W gives -1 in every plane.
 * n may be 0 (nothing is enqueued).
 */
int ih_query_rect(const int32_t *ih, int32_t P, int32_t H, int32_t W,
                  int32_t layout, const ih_rect *rects, int64_t n,
                  int32_t *out, void *stream);

/*
 * ih_query_weighted - spatially weighted local histograms (Eq. 3.1) with the
 * Manhattan kernel (Eq. 3.3), in O(1) per window by SWIH (Sec. 3.1.3): the
 * kernel is split into quadrants in which the weight is affine in the pixel
 * coordinates, and each quadrant is read from the count and moment integral
 * histograms (Eq. 3.4) and translated to the window centre.
 *
 * Weight of pixel (x, y) in a window of h rows and w columns (the thesis
 * gives no constants; this is the reading used):
 *   w(x,y) = 1 - ( |x - xc| / (h/2) + |y - yc| / (w/2) ) / 2,
 *   xc = (r0 + r1 - 1) / 2,  yc = (c0 + c1 - 1) / 2,
 * so that w = N(x,y) / (2hw) with the integer
 *   N(x,y) = 2hw - w |2x - (r0+r1-1)| - h |2y - (c0+c1-1)|.
 * out(q, p) = sum over the window's pixels of plane p of N, as an exact
 * int64, divided in FP64 by 2hw (or, when l1_normalize is non-zero, by the
 * sum of N over the whole window, making each channel sum to 1), rounded to
 * FP32.
 *
 *   ih, mom_x, mom_y  device, from ih_build with moments, in `layout`.
 *   P, H, W, C        their shape; P must be a multiple of C.
 *   rects             device, n windows.
 *   kernel            IH_MANHATTAN.
 *   out               device, out: n x P float.  Empty windows give zeros;
 *                     windows outside the frame, or with h * w * max(r1, c1)
 *                     >= 2^32 (where moment sums could wrap), give NaN.
 */
int ih_query_weighted(const int32_t *ih, const uint32_t *mom_x,
                      const uint32_t *mom_y, int32_t P, int32_t H, int32_t W,
                      int32_t C, int32_t layout, const ih_rect *rects,
                      int64_t n, int32_t kernel, int32_t l1_normalize,
                      float *out, void *stream);

/*
 * ih_pyramid_desc - spatial-pyramid region descriptors (Alg. 2 with the
 * concatenated layout of Sec. 2.4.4).  Level l (0 <= l < levels) splits the
 * window into 2^l x 2^l cells; cell (i, j) of window {r, c, h, w} covers
 * rows [r + floor(i h / 2^l), r + floor((i+1) h / 2^l)) and likewise columns.
 * The descriptor of a window is the concatenation, level by level (coarse
 * first), of its cells in row-major order, each holding P int32 counts:
 * cells(levels) = sum_l 4^l (1, 5, 21, 85) cells.
 *   wins   device, n x 4 int32 {r, c, h, w}.
 *   levels 1..4.
 *   out    device, out: n x cells x P int32; windows not inside the frame
 *          (h < 1, w < 1, r < 0, c < 0, r + h > H or c + w > W) give -1.
 */
int ih_pyramid_desc(const int32_t *ih, int32_t P, int32_t H, int32_t W,
                    int32_t layout, const int32_t *wins, int64_t n,
                    int32_t levels, int32_t *out, void *stream);

/*
 * ih_match_candidates - exhaustive sliding-window search (Sec. 2.4.3): the
 * pyramid descriptor of every candidate window {origins[i], win_h, win_w} is
 * compared with a template descriptor and the best candidate is selected.
 * Distances sum over levels with the pyramid-match weights of Eq. 2.24
 * (level 0: 1/2^L, level l >= 1: 1/2^(L-l+1), L = levels - 1):
 *   IH_CHI2: sum (a-b)^2 / (a+b) over cells and planes, 0/0 := 0, on raw
 *            counts (the thesis does not define chi-square; reading used);
 *            per-term FP32, accumulated in FP64;
 *   IH_L1:   sum |a-b| (Eq. 2.22, p = 1), exact integer arithmetic;
 *   IH_PMK:  sum min(a,b) (Eq. 2.23), a similarity, exact integer arithmetic.
 *   tmpl_desc  device, cells(levels) x P int32 template descriptor, as
 *              written by ih_pyramid_desc.
 *   origins    device, n x 2 int32 (row, column) candidate origins.
 *   dist       device, out: n floats.  Candidates not fully inside the frame
 *              get +inf (CHI2, L1) or -inf (PMK).
 *   best       device, out: one int32, the lowest candidate index with the
 *              smallest distance (largest similarity for IH_PMK), or -1 if
 *              no candidate lies inside the frame.
 * IH_ERR_RANGE when n >= 2^31 or, planes innermost, W * P >= 2^32.
 */
int ih_match_candidates(const int32_t *ih, int32_t P, int32_t H, int32_t W,
                        int32_t layout, const int32_t *tmpl_desc,
                        int32_t win_h, int32_t win_w, int32_t levels,
                        const int32_t *origins, int64_t n, int32_t metric,
                        float *dist, int32_t *best, void *stream);

/*
 * Batched build and search over many frames of uneven size and bin count
 * (the device-resident analogue of the thesis's dual-buffered frame
 * pipeline, Alg. 10): every frame's integral histogram (in its layout),
 * optionally its template descriptor and its candidate search (3-level
 * pyramid, as ih_pyramid_desc / ih_match_candidates), over all frames at
 * once.  The calls allocate nothing and do not synchronise; the phased mode
 * may be captured in a HIP graph and replayed.
 */
typedef struct {
  const void *img;          /* device, C x H x W values of the batch dtype   */
  int32_t *ih;              /* device, out: P x H x W (IH_BHW) or H x W x P
                               (IH_HWB) int32                               */
  int32_t H, W, C, bins, value_bits;
  ih_tile_cfg tile;         /* tile shape; tile_h == 0 selects the heuristic.
                               IH_BHW: planes_per_wave 1, 2, 4 or 8         */
  /* candidate search; n_cand == 0 skips it for this frame                   */
  const int32_t *tmpl_desc; /* device, 21 x P template descriptor, or NULL to
                               compute it from tmpl_win of this frame       */
  int32_t tmpl_win[4];      /* {r, c, h, w}, used when tmpl_desc is NULL     */
  int32_t *tmpl_out;        /* device, out: 21 x P, when tmpl_desc is NULL   */
  int32_t win_h, win_w;     /* candidate window                              */
  const int32_t *origins;   /* device, n_cand x 2 (row, column)              */
  int64_t n_cand;
  float *dist;              /* device, out: n_cand distances                 */
  int32_t *best;            /* device, out: best candidate index or -1       */
  int32_t layout;           /* ih_layout of this frame's histogram           */
} ih_frame;

/* Bytes of the plan for n frames (0 when n < 1). */
size_t ih_batch_plan_bytes(int32_t n);

/*
 * ih_batch_plan - host-only: validate n frames, choose their tile shapes and
 * work ranges, and write the plan (plan_bytes >= ih_batch_plan_bytes(n)).
 * dtype (IH_U8 / IH_U16) and metric (IH_CHI2 / IH_L1 / IH_PMK) are shared by
 * the batch.  *ws_bytes receives the workspace size ih_build_batch needs.  The
 * caller copies the plan to device memory once; it stays valid for every
 * launch with the same frames and buffers.
 */
int ih_batch_plan(const ih_frame *frames, int32_t n, int32_t dtype,
                  int32_t metric, void *plan, size_t plan_bytes,
                  size_t *ws_bytes);

/* How ih_build_batch runs a plan. */
typedef enum {
  IH_BATCH_PHASED = 0,      /* one launch per phase, each over all frames   */
  IH_BATCH_COOPERATIVE = 1  /* one cooperative persistent launch; phases are
                               separated by the runtime's grid barrier       */
} ih_batch_mode;

/*
 * ih_build_batch - enqueue the batch described by a plan.
 *   plan_host  the plan as written by ih_batch_plan (host memory).
 *   plan_dev   a device copy of the same bytes.
 *   ws         device workspace of ws_bytes (contents on entry do not matter).
 *   mode       ih_batch_mode; both produce identical results.
 * Phases: tile histograms, carry scans, write-out, template descriptors,
 * candidate scoring, best candidate; each phase of a frame depends only on
 * earlier phases of the same frame.  The phased mode allocates no memory,
 * synchronises nothing and may be captured in a HIP graph.  When the plan has
 * frames of several write-out classes (bin-major tiles, bin-major strips,
 * planes innermost, planes innermost in column streams), the write-out phase
 * runs each class's kernel as a branch of its own, and so does the scoring
 * phase for each layout when the plan has both: the first on stream, the
 * others on up to three auxiliary streams (default priority) that the
 * library creates once per device, on the first call whose stream is not
 * being captured, and keeps until the process ends; the branches are forked
 * from and joined back into stream with events, so all work stays ordered
 * with stream.  Before those streams exist the classes run one after another
 * on stream.  Every call on a device shares them: the enqueueing of that
 * phase is serialised between host threads, and a call on one thread while
 * another thread captures a batch on the same device may fail with an
 * error.  The cooperative
 * mode returns IH_ERR_UNSUPPORTED, enqueuing nothing, when the stream is
 * capturing: a captured cooperative launch becomes a plain kernel node whose
 * grid barrier has no co-residency guarantee.
 */
int ih_build_batch(const void *plan_host, const void *plan_dev, void *ws,
                   size_t ws_bytes, int32_t mode, void *stream);

/*
 * ih_build_moments2 - second coordinate-moment integral histograms (the
 * weighted integral histograms of Eq. 3.4 for the weights x^2 and y^2):
 *   Mxx(p,r,c) = sum over r' <= r, c' <= c of r'^2 * [bin(r',c') = p]
 *   Myy(p,r,c) = sum over r' <= r, c' <= c of c'^2 * [bin(r',c') = p]
 * stored modulo 2^32, by two builds with coordinate weights.  With the count
 * and moment tensors of ih_build they give the quadratic kernel in O(1)
 * (ih_query_quadratic).
 *   img, dtype, H, W, C, bins, value_bits, layout, cfg, ws, ws_bytes, stream
 *               as for ih_build (workspace: ih_build_workspace_size with
 *               moments = 0).
 *   mom_xx, mom_yy  device, out: P x H x W uint32 each (in layout).
 * Returns IH_OK or IH_ERR_*.
 */
int ih_build_moments2(const void *img, int32_t dtype, int32_t H, int32_t W,
                      int32_t C, int32_t bins, int32_t value_bits,
                      int32_t layout, uint32_t *mom_xx, uint32_t *mom_yy,
                      const ih_tile_cfg *cfg, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * ih_query_quadratic - spatially weighted local histograms (Eq. 3.1) with the
 * quadratic kernel of the squared Euclidean distance (Fig. 3.1), exact in
 * O(1) per window: the weight is a combination of 1, x, x^2, y, y^2, each
 * read over the window from its integral histogram (Eq. 3.4, Eq. 2.16) and
 * combined about the window centre (the SWIH steps of Sec. 3.1.3; this
 * kernel needs no quadrant split).
 *
 * Weight of pixel (x, y) in a window of h rows and w columns, in normalised
 * coordinates u = (x - xc) / (h/2), v = (y - yc) / (w/2) with
 * xc = (r0 + r1 - 1) / 2, yc = (c0 + c1 - 1) / 2:
 *   K = 1 - (u^2 + v^2) / 2 = N2 / (2 h^2 w^2),
 *   N2 = 2 h^2 w^2 - w^2 (2x - (r0+r1-1))^2 - h^2 (2y - (c0+c1-1))^2.
 * out(q, p) = the sum of N2 over the window's pixels of plane p, an exact
 * int64, divided in FP64 by 2 h^2 w^2 (or, with l1_normalize, by the sum of
 * N2 over the whole window), rounded to FP32.
 *
 *   ih, mom_x, mom_y   device, from ih_build with moments, in `layout`.
 *   mom_xx, mom_yy     device, from ih_build_moments2, in `layout`.
 *   P, H, W, C, layout, rects, n, out, stream  as for ih_query_weighted.
 * Empty windows give zeros; windows outside the frame, or so large that
 * w (h-1) h (2h-1) / 6 or h (w-1) w (2w-1) / 6 reaches 2^32, give NaN.
 */
int ih_query_quadratic(const int32_t *ih, const uint32_t *mom_x,
                       const uint32_t *mom_y, const uint32_t *mom_xx,
                       const uint32_t *mom_yy, int32_t P, int32_t H,
                       int32_t W, int32_t C, int32_t layout,
                       const ih_rect *rects, int64_t n, int32_t l1_normalize,
                       float *out, void *stream);

/*
 * ih_query_wedding - the wedding-cake approximation of a spatially weighted
 * local histogram (Eq. 3.2, Sec. 3.1.2), from the count integral histogram.
 * Layer j = 1..layers of a window with h rows and w columns is the centred
 * window with margins floor((layers-j) h / (2 layers)) rows and
 * floor((layers-j) w / (2 layers)) columns (layer `layers` is the window);
 * ring j (layer j minus layer j-1) is weighted by the kernel's mean over the
 * ring in normalised coordinates (the kernel as for ih_query_quadratic:
 * IH_MANHATTAN 1 - (|u|+|v|)/2, IH_QUADRATIC 1 - (u^2+v^2)/2, IH_GAUSSIAN
 * exp(-(u^2+v^2) / (2 sigma^2))).  The sum over rings of weight times ring
 * count is taken in FP64 and rounded to FP32, on the same scale as the
 * exact kernels' non-normalised output.
 *   layers   1..16;  sigma  > 0 for IH_GAUSSIAN (relative to the half-sizes).
 *   Other arguments as for ih_query_weighted; empty windows give zeros,
 *   windows outside the frame NaN.
 */
int ih_query_wedding(const int32_t *ih, int32_t P, int32_t H, int32_t W,
                     int32_t C, int32_t layout, const ih_rect *rects,
                     int64_t n, int32_t layers, int32_t kernel, double sigma,
                     float *out, void *stream);

/*
 * ih_color_likelihood - FG/BG colour likelihood map (Sec. 2.4.2,
 * Eq. 2.18-2.21).  Joint RGB histograms with 32 x 32 x 32 bins (bin =
 * ((R>>3)*32 + (G>>3))*32 + (B>>3)) of the foreground rectangle fg and of
 * the background rectangle bg minus fg (Eq. 2.18); every pixel's likelihood
 * of belonging to the foreground is
 *   L = H_FG(b) / (H_FG(b) + H_BG(b))   (Eq. 2.21; 0 where both are 0),
 * and its 8-bit code is q = round-half-up(255 L), computed in integers as
 * (510 H_FG + T) / (2 T), T = H_FG + H_BG.
 *   rgb      device, 3 x H x W uint8 (R, G, B planes), H * W < 2^31.
 *   fg, bg   rectangles (by value, half-open) inside the image.
 *   ws       device workspace of ws_bytes >= ih_color_likelihood_workspace_size().
 *   q        device, out: H x W uint8 codes.
 *   L        device, out: H x W float likelihoods (FP64 ratio rounded to
 *            FP32), or NULL.
 * Returns IH_OK or IH_ERR_*.
 */
size_t ih_color_likelihood_workspace_size(void);
int ih_color_likelihood(const uint8_t *rgb, int32_t H, int32_t W, ih_rect fg,
                        ih_rect bg, void *ws, size_t ws_bytes, uint8_t *q,
                        float *L, void *stream);

/*
 * ih_moment_images - moment integral images of an 8-bit map q (the zero and
 * first moments of Alg. 1 over any rectangle in O(1)):
 *   S(r,c)  = sum over r' <= r, c' <= c of q(r',c')          (int32, exact)
 *   Sx(r,c) = sum of r' * q(r',c'),  Sy(r,c) = sum of c' * q(r',c')
 *             (uint32, modulo 2^32)
 * built by one integral-histogram build with one plane, the weights q and
 * moments.
 *   q           device, H x W uint8; H * W * 255 <= 2^31 - 1.
 *   S, Sx, Sy   device, out: H x W each.
 *   cfg, ws, ws_bytes  as for ih_build with C = 1, bins = 1, IH_BHW and
 *               moments (workspace: ih_build_workspace_size(H, W, 1, 1, 1,
 *               IH_BHW, cfg)).
 * Returns IH_OK or IH_ERR_*.
 */
int ih_moment_images(const uint8_t *q, int32_t H, int32_t W, int32_t *S,
                     uint32_t *Sx, uint32_t *Sy, const ih_tile_cfg *cfg,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * ih_camshift - CAMSHIFT (Alg. 1) from many start points at once on moment
 * integral images (one thread per start).  Each step places the fixed
 * win_h x win_w search window at r0 = floor(cr - (win_h-1)/2 + 0.5),
 * c0 = floor(cc - (win_w-1)/2 + 0.5), shifted inside the image, reads its
 * M00 and first moments from S, Sx, Sy (four corners each), and moves the
 * centre to the centroid (row moment / M00, column moment / M00, in FP64).
 * It stops when the squared move is below delta^2, when M00 = 0 (the centre
 * stays), or after max_iter steps.
 *   S, Sx, Sy   device, from ih_moment_images.
 *   starts      device, n x 2 double (row, column).
 *   win_h, win_w  window, at most the image; 255 w h (h-1) / 2 and
 *               255 h w (w-1) / 2 must be below 2^32 (IH_ERR_RANGE).
 *   centers     device, out: n x 2 double;  iters  device, out: n int32.
 * Returns IH_OK or IH_ERR_*; n may be 0.
 */
int ih_camshift(const int32_t *S, const uint32_t *Sx, const uint32_t *Sy,
                int32_t H, int32_t W, const double *starts, int64_t n,
                int32_t win_h, int32_t win_w, double delta, int32_t max_iter,
                double *centers, int32_t *iters, void *stream);

/*
 * ih_jih_update - joint integral histogram update of the spatio-temporal
 * median (Alg. 4, Fig. 4.1): JIH = JIH + IH(head) - IH(tail), in place.
 * The joint IH of a window of frames is the integral histogram of all their
 * pixels; sliding the window by one frame adds the entering (head) frame and
 * removes the leaving (tail) one.  Computed as one build of the integral
 * histogram of the difference (head +1, tail -1 per pixel, modulo 2^32)
 * whose write-out adds into jih, so each update reads and writes jih once.
 * The planes are stored cumulative over each channel's bins: plane
 * ch*bins + k holds the counts of bins 0..k (the plain count of bin k is the
 * difference of planes k and k-1).
 *
 *   head        device, C x H x W values of type dtype: the entering frame.
 *   tail        device, same shape and dtype: the leaving frame, or NULL
 *               while the window is filling (then JIH = JIH + IH(head)).
 *   dtype, H, W, C, bins, value_bits, layout, cfg, ws, ws_bytes, stream
 *               as for ih_build, except that cfg = NULL selects the update's
 *               own default tile (workspace: ih_jih_update_workspace_size).
 *               IH_HWB needs P <= 512 and tile_w * P <= 16384.
 *   jih         device, in/out: P x H x W int32 (in layout), cumulative
 *               planes.  Start from zeros.  Every entry stays exact while
 *               the window's frame count * H * W < 2^31.
 * Returns IH_OK or IH_ERR_*.  jih must not overlap the frames or ws.
 */
size_t ih_jih_update_workspace_size(int32_t H, int32_t W, int32_t C,
                                    int32_t bins, int32_t layout,
                                    const ih_tile_cfg *cfg);
int ih_jih_update(const void *head, const void *tail, int32_t dtype,
                  int32_t H, int32_t W, int32_t C, int32_t bins,
                  int32_t value_bits, int32_t layout, int32_t *jih,
                  const ih_tile_cfg *cfg, void *ws, size_t ws_bytes,
                  void *stream);

/*
 * ih_local_median - per-pixel median of the spatio-temporal box from a joint
 * integral histogram (Alg. 4, ComputeLocalMedian; Sec. 4.1.1).
 *   jih         device, P x H x W int32 (in layout), P = C * bins, the
 *               cumulative planes of ih_jih_update holding exactly `frames`
 *               frames.  The median is found by a binary search over the
 *               cumulative counts (bin-major) or 64 bins at a time
 *               (planes innermost).
 *   frames      number of frames in the window (T + 1), >= 1.
 *   win_h, win_w  spatial window; pixel (r, c) uses rows
 *               r - (win_h-1)/2 .. r + win_h/2 and columns likewise,
 *               clipped to the image.
 *   median      device, out: C x H x W int32 bin indices.  The median of the
 *               N = frames * (window area) samples is the first bin whose
 *               running count reaches ceil(N/2) (the lower median for even N).
 * Needs bins <= 256 and frames * H * W < 2^31.  A jih that does not hold
 * `frames` frames gives unspecified (in-bounds) bins.  Returns IH_OK or
 * IH_ERR_*.
 */
int ih_local_median(const int32_t *jih, int32_t C, int32_t bins, int32_t H,
                    int32_t W, int32_t layout, int32_t frames, int32_t win_h,
                    int32_t win_w, int32_t *median, void *stream);

/*
 * ih_build_passes - the number of passes (1 or 3) ih_build uses for a
 * layout and configuration (cfg may be NULL), or IH_ERR_INVALID_ARG.
 */
int ih_build_passes(int32_t layout, const ih_tile_cfg *cfg);

/*
 * ih_set_lookback_patience - look-back policy of the single-pass build
 * (IH_PASSES_ONE), for every later build in this process.  Before each
 * tile's look-back, a band worker polls the flag of the band directly above
 * at most `polls` times for its inclusive bottom row; then (or at once for
 * polls <= 0, the default -1 included) it takes the nearest inclusive row
 * published above plus the aggregates of the bands in between.  Results are
 * identical for every value; only the time differs.  Returns IH_OK, or
 * IH_ERR_INVALID_ARG for polls < -1.
 */
int ih_set_lookback_patience(int32_t polls);

/*
 * ih_profile_events - profiling hook.  When both are non-NULL (hipEvent_t),
 * every later build on this thread (ih_build, ih_build_weighted,
 * ih_build_moments2, ih_jih_update) records `start` on its stream just
 * before its dominant kernel (the final write-out of a three-pass build, the
 * band kernel of a single-pass one) and `stop` just after it, so that the
 * caller can time that kernel alone.  Passing NULL, NULL turns it off.
 */
int ih_profile_events(void *start, void *stop);

#ifdef __cplusplus
}
#endif

#endif /* IH_H */
