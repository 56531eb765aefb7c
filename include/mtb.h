/*
 * mtb.h -- C ABI of libmtb, Median Threshold Bitmap (MTB) translational
 * alignment of exposure stacks on AMD Instinct MI355X (gfx950).
 *
 * The method is Ward's MTB alignment as accelerated in Alpay, Aydemir and
 * Akyuz, "Accelerating Translational Image Registration for HDR Images on
 * GPU" (arXiv 2007.06483): gray conversion, a 2x pyramid, a per-level
 * 256-bin histogram median, threshold and exclusion bitmaps, and a
 * coarse-to-fine search over the nine +-1 shifts at each level that scores a
 * shift by XOR/AND-ing the bitmaps and counting the set pixels
 * (Section III-A; Section III-B; Fig. 2).
 *
 * Conventions for every call:
 *   - Memory.  Every pointer named d_* is device memory owned by the caller;
 *     the library allocates no device memory and keeps no state between
 *     calls apart from the launch-shape table that mtb_tune_stack and
 *     mtb_set_shape fill (it changes speed, never results).  Host arrays are
 *     named h_*.
 *   - Streams.  `stream` is a hipStream_t passed as void* (NULL is the null
 *     stream).  All device work is enqueued on it and runs asynchronously;
 *     results are valid once the stream has reached the call's work.
 *   - Errors.  Arguments are validated before anything is enqueued; on a
 *     validation error (MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE,
 *     MTB_ERR_UNSUPPORTED) nothing has been enqueued.  A failed kernel launch
 *     returns MTB_ERR_DEVICE: kernels enqueued before it still run and the
 *     call's outputs are undefined, and the next call on the same buffers
 *     starts afresh.  No call aborts or throws.
 *   - Images.  An RGB image is `height` rows of `width` interleaved R,G,B
 *     bytes; row y starts at byte y * row_stride (row_stride >= 3 * width).
 *     width * height must be below 2^31.
 *   - Levels.  Level l of a width x height image is (width >> l) x
 *     (height >> l); level 0 is full resolution.  1 <= levels <=
 *     mtb_max_levels(width, height).  The search reaches shifts of up to
 *     +-(2^levels - 1) pixels per axis.
 *   - Shifts.  A shift (dx, dy) is what to apply to the moving image to align
 *     it with the reference: aligned[y][x] = moving[y - dy][x - dx].
 *   - Thread safety.  Calls are reentrant and may come from several host
 *     threads at once (the shared caches and the shape table are guarded);
 *     calls on one stream that share a buffer are ordered by the stream.
 */
#ifndef MTB_H
#define MTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTB_MAX_LEVELS 16 /* width * height < 2^31 allows at most 16 levels */
#define MTB_MAX_STACK 32  /* images per mtb_align_stack call */

typedef enum mtb_status {
    MTB_OK = 0,
    MTB_ERR_INVALID_ARG = 1, /* null pointer, size or level out of range, ... */
    MTB_ERR_WORKSPACE = 2,   /* a buffer is smaller than its *_bytes query */
    MTB_ERR_DEVICE = 3,      /* HIP reported an error while enqueuing */
    MTB_ERR_UNSUPPORTED = 4  /* no usable gfx950 device */
} mtb_status;

/*
 * Where everything lives inside the two per-image buffers.  All offsets are
 * in bytes from the start of their buffer and are multiples of 256.
 *
 * Pyramid buffer (written by mtb_build_pyramid):
 *   gray level l: level_height[l] rows of gray_pitch[l] bytes at gray_offset[l];
 *     byte x of row y is the gray value of pixel (x, y) for x < level_width[l]
 *     (the bytes past level_width[l] are padding with no defined value);
 *   histogram: uint32 hist[levels][256] at hist_offset (Section III-B);
 *   the bytes from the end of the histogram to pyramid_bytes are scratch the
 *   build uses while merging histograms, with no defined value afterwards.
 * Bitmaps buffer (written by mtb_bitmaps):
 *   the first 256 bytes are a guard with no defined value;
 *   level l threshold bitmap T and exclusion bitmap E: each level_height[l]
 *     rows of words_per_row[l] uint64 words at tb_offset[l] / eb_offset[l];
 *     pixel x of row y is bit (x % 64) of word (x / 64) of the row (least
 *     significant bit first); bits past level_width[l] are 0 (rows are
 *     padded to a multiple of 128 pixels);
 *   medians: int32 median[levels] at median_offset.
 */
typedef struct mtb_layout {
    int32_t width, height, levels;
    int32_t level_width[MTB_MAX_LEVELS];
    int32_t level_height[MTB_MAX_LEVELS];
    int32_t words_per_row[MTB_MAX_LEVELS]; /* 2 * ceil(level_width / 128) */
    int64_t gray_offset[MTB_MAX_LEVELS];
    int64_t gray_pitch[MTB_MAX_LEVELS]; /* 64 * words_per_row */
    int64_t hist_offset;
    int64_t pyramid_bytes;
    int64_t tb_offset[MTB_MAX_LEVELS];
    int64_t eb_offset[MTB_MAX_LEVELS];
    int64_t median_offset;
    int64_t bitmaps_bytes;
} mtb_layout;

/* Human-readable name of a status code (static storage; never NULL). */
const char *mtb_status_string(mtb_status status);

/* Largest level count L with (width >> (L-1)) >= 1 and (height >> (L-1)) >= 1;
 * 0 if width or height is below 1. */
int32_t mtb_max_levels(int32_t width, int32_t height);

/* Fills *out with the buffer layout for the given size and level count.
 * MTB_ERR_INVALID_ARG if out is NULL or the size or level count is out of range. */
mtb_status mtb_get_layout(int32_t width, int32_t height, int32_t levels, mtb_layout *out);

/* Bytes of one image's pyramid buffer / bitmaps buffer; 0 if the arguments are invalid. */
size_t mtb_pyramid_bytes(int32_t width, int32_t height, int32_t levels);
size_t mtb_bitmaps_bytes(int32_t width, int32_t height, int32_t levels);

/* Bytes of the workspace mtb_align_pair needs (search counters); 0 if levels is out of range. */
size_t mtb_pair_workspace_bytes(int32_t levels);

/* Bytes of the workspace mtb_align_stack needs for n images; 0 if invalid. */
size_t mtb_stack_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t levels);

/*
 * Where mtb_align_stack (and the chained mode) leave each image's pyramid
 * buffer and bitmaps buffer (layouts as described at mtb_layout) inside a
 * workspace at d_workspace: h_pyramids[i] and h_bitmaps[i] receive device
 * addresses inside that workspace, for i < n.  Nothing is read or written on
 * the device.  Where mtb_level1_from_level0 says so, the alignment calls form
 * level 1's bitmaps from level 0's gray and do not store level 1's gray
 * (mtb_build_pyramid always does); every other part of both layouts is
 * filled in.
 * Errors: MTB_ERR_INVALID_ARG (null pointers, n, sizes or levels out of range).
 */
mtb_status mtb_stack_image_buffers(const void *d_workspace, int32_t n, int32_t width, int32_t height,
                                   int32_t levels, void **h_pyramids, void **h_bitmaps);

/*
 * Whether the alignment calls, for a launch set of n images of this size,
 * form level 1's bitmaps from level 0's gray and leave level 1's gray out of
 * the workspace (1) or store it (0), under the shape stored for that key
 * (see mtb_launch_shape) or the built-in rule.  -1 for arguments out of range.
 */
int32_t mtb_level1_from_level0(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels);

/*
 * Gray pyramid and per-level histograms of one RGB image (Section III-A:
 * gray conversion and the 2x pyramid; Section III-B: 256-bin histograms of
 * every level).  gray = (54 R + 183 G + 19 B) >> 8; each coarser level is the
 * floor mean of 2x2 blocks of the level below, an odd last row or column
 * being dropped.
 *   d_rgb            device RGB image (see Images above)
 *   d_pyramid        device buffer of pyramid_bytes >= mtb_pyramid_bytes(...)
 *                    receiving the layout described at mtb_layout
 * Errors: MTB_ERR_INVALID_ARG (null pointer, sizes, stride, levels),
 *         MTB_ERR_WORKSPACE (pyramid_bytes too small), MTB_ERR_DEVICE.
 */
mtb_status mtb_build_pyramid(const uint8_t *d_rgb, int32_t width, int32_t height,
                             int64_t row_stride, int32_t levels, void *d_pyramid,
                             size_t pyramid_bytes, void *stream);

/*
 * Medians and threshold / exclusion bitmaps of every level of a pyramid
 * (Section III-A: median threshold; Section III-B: median per histogram and
 * exclusion bitmaps).  m = lower median of the level (element (P-1)/2 of its
 * sorted P pixels); T = [g > m]; E = [|g - m| > exclude_range].
 *   d_pyramid        a pyramid buffer written by mtb_build_pyramid (same size/levels)
 *   exclude_range    half-width of the excluded band around the median, 0..255 (Ward: 4)
 *   d_bitmaps        device buffer of bitmaps_bytes >= mtb_bitmaps_bytes(...)
 * Errors: MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
mtb_status mtb_bitmaps(const void *d_pyramid, int32_t width, int32_t height, int32_t levels,
                       int32_t exclude_range, void *d_bitmaps, size_t bitmaps_bytes,
                       void *stream);

/*
 * Coarse-to-fine shift search between two images' bitmaps (Section III-A:
 * +-1 tests per level, doubling between levels; Section III-B: XOR of the
 * threshold bitmaps, AND of both exclusion bitmaps, count of set pixels).
 * Starting from (0, 0) at the coarsest level, each level tests the nine
 * shifts base + (ddx, ddy), ddx, ddy in {-1, 0, 1}; the error of shift c is
 *   e(c) = #{(x, y) : (T_ref ^ S_c T_mov) & E_ref & S_c E_mov}
 * with (S_c B)[y][x] = B[y - cy][x - cx], zero where that falls outside the
 * image.  The lowest error wins, ties going to the lowest (ddy, ddx)
 * (ddy-major order); the next level's base is twice the winner.
 * A pair whose two bitmaps buffers' planes fit 144 KiB is searched by one
 * workgroup in one launch that leaves the workspace untouched; larger pairs
 * take a zeroing launch, the coarse levels' launch and one launch per finer
 * level, with their counters in the workspace.
 *   d_bm_ref, d_bm_mov   bitmaps buffers written by mtb_bitmaps
 *   d_workspace          >= mtb_pair_workspace_bytes(levels) bytes, contents ignored
 *   d_shift              int32[2] receives (dx, dy) at level 0
 *   d_err                uint32[1] receives the level-0 error of that shift
 *   d_trace              NULL or uint32[levels][9]: error of candidate
 *                        (ddy + 1) * 3 + (ddx + 1) at each level
 *   d_level_shifts       NULL or int32[levels][2]: the shift chosen at each level
 * Errors: MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
mtb_status mtb_align_pair(const void *d_bm_ref, const void *d_bm_mov, int32_t width,
                          int32_t height, int32_t levels, void *d_workspace,
                          size_t workspace_bytes, int32_t *d_shift, uint32_t *d_err,
                          uint32_t *d_trace, int32_t *d_level_shifts, void *stream);

/*
 * mtb_align_pair without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the search state (counters, bases,
 * coarse surfaces, tickets; at most 30720 bytes, enough for MTB_MAX_LEVELS
 * levels) lives in a static device array of the library, one per device,
 * held until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); it clears the array with a kernel
 * before the search (a pair searched by one workgroup, as in mtb_align_pair,
 * neither clears nor uses it).  Every call on a device shares that device's array and
 * leaves its last contents there: calls that overlap on one device (on
 * different streams or host threads) race and must be ordered by the caller.
 * Arguments, results and errors as for mtb_align_pair, minus the workspace;
 * MTB_ERR_WORKSPACE if the state of `levels` levels would not fit the array
 * (never for valid levels), MTB_ERR_DEVICE if the array's address cannot be
 * obtained.
 */
mtb_status mtb_align_pair_scratch(const void *d_bm_ref, const void *d_bm_mov, int32_t width,
                                  int32_t height, int32_t levels, int32_t *d_shift, uint32_t *d_err,
                                  uint32_t *d_trace, int32_t *d_level_shifts, void *stream);

/*
 * Whole-stack alignment (Section III-B: every image is uploaded once, its
 * pyramid and bitmaps computed once, and the stack aligned pairwise).  Every
 * image is aligned against the reference image; each image's pyramid,
 * histograms, medians and bitmaps are built once, and all pairs share the
 * reference's.  The reference reports shift (0, 0) and error 0.
 *   h_d_rgb          host array of n device pointers, one RGB image each (same size and stride)
 *   n                1 .. MTB_MAX_STACK
 *   ref_index        index of the reference, or -1 for n / 2
 *   exclude_range    as for mtb_bitmaps (Ward: 4)
 *   d_workspace      >= mtb_stack_workspace_bytes(n, width, height, levels) bytes
 *   d_shifts         int32[n][2] receives (dx, dy) per image
 *   d_errs           uint32[n] receives each image's level-0 error
 *   d_trace          NULL or uint32[n][levels][9] (as for mtb_align_pair; zeros for the reference)
 * Errors: MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
mtb_status mtb_align_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                           int32_t height, int64_t row_stride, int32_t levels,
                           int32_t exclude_range, int32_t ref_index, void *d_workspace,
                           size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                           uint32_t *d_trace, void *stream);

/*
 * The paper's representation, for comparison (Section III-B: T and E kept as
 * one byte per pixel, 255 or 0, instead of bit-packed words).  Same results
 * as mtb_align_stack — the error counts do not depend on the representation —
 * through a byte-map pass and a byte-map search over every level (no
 * exhaustive coarse windows).  Arguments as for mtb_align_stack, with a
 * workspace of mtb_stack_bytemaps_workspace_bytes(n, width, height, levels).
 */
size_t mtb_stack_bytemaps_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t levels);
mtb_status mtb_align_stack_bytemaps(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                                    int32_t height, int64_t row_stride, int32_t levels,
                                    int32_t exclude_range, int32_t ref_index, void *d_workspace,
                                    size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                                    uint32_t *d_trace, void *stream);

/*
 * Chained stack alignment (Section III-A: consecutive exposures are the ones
 * compared; Section III-B: a stack of n images takes n - 1 pairwise
 * alignments).  Image i is aligned against its neighbour towards the
 * reference (i + 1 below it, i - 1 above), whose exposure is closest to its
 * own, and the pairwise shifts are summed along the chain, translations
 * composing by addition.  Arguments and buffers as for mtb_align_stack;
 * d_shifts receives the summed shift of each image against the reference,
 * d_errs and d_trace the pairwise level-0 errors and traces.
 */
mtb_status mtb_align_stack_chained(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                                   int32_t height, int64_t row_stride, int32_t levels,
                                   int32_t exclude_range, int32_t ref_index, void *d_workspace,
                                   size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                                   uint32_t *d_trace, void *stream);

/*
 * Launch shapes and their tuner.  How an alignment is cut into workgroups
 * never changes its results (every shape gives the same bits); it changes
 * its speed, and the best shape depends on the image size and count.  A
 * shape (mtb_launch_shape) fixes:
 *   - the pyramid pass: workgroups as a percentage of one round of the
 *     workgroups the device holds at once, and how many horizontally
 *     adjacent 64x256 tiles a workgroup takes at a time (1, 2 or 4);
 *   - the bitmaps pass: workgroups as a percentage of one resident round, and
 *     wavefronts per workgroup (2, 4 or 8);
 *   - the search: how many of the coarsest levels are searched over
 *     exhaustive windows (radius 1, 3, 7, 15, 31 from the coarsest down;
 *     -1: the built-in rule, up to three levels of at most 8192 words of
 *     32 bits; 0..5; the results are the same either way),
 *     and per fine level the rows each row stream covers
 *     and the lanes of a row stream (8, 16, 32 or 64; 0: the built-in rules,
 *     the fewest rows that keep one level's grid within one resident round
 *     and the width that pads rows least); and whether a pair whose two
 *     bitmap pyramids fit 144 KiB (every plane of the bitmaps buffer, from
 *     the end of its leading 256-byte guard to the medians) is searched by one
 *     workgroup that holds both in LDS and runs every level in one launch
 *     (-1 or 1, the default) or by the launches above (0); and whether the
 *     bitmaps pass forms level 1's bitmaps from level 0's gray, two rows at a
 *     time, so that the pyramid pass need not store level 1's gray (1), or
 *     stores and reads level 1's gray like every other level (0); the
 *     built-in rule (-1) takes the first for launch sets of at least 96 Mi
 *     level-0 pixels (n * width * height), where the 2 x 25 % of a level's
 *     traffic it saves outweighs the bitmaps pass's second median per
 *     wavefront.  Results are identical either way.
 * Shapes are kept per key (n images, width, height, levels, and whether
 * row_stride is a multiple of 16, else of 4, else neither) in a process-wide
 * table guarded by a mutex.  A key without a shape of its own uses the shape
 * last stored for its bucket: same n, levels and row-stride class, and a
 * pixel count in the same half octave (round(2 log2(width * height))).
 * mtb_align_stack, mtb_align_stack_chained and, per group of equal items,
 * mtb_align_batch and mtb_align_quadrants use the table's shape, the
 * built-in shape otherwise.
 */
typedef struct mtb_launch_shape {
    int32_t pyramid_slots_pct;  /* 25 .. 400 (default 100) */
    int32_t pyramid_tile_group; /* 1, 2 or 4 (default 1) */
    int32_t bitmaps_blocks_pct; /* 25 .. 100 (default 100) */
    int32_t bitmaps_waves;      /* 2, 4 or 8 (default 4) */
    int32_t coarse_levels;      /* -1 (rule), 0 .. 5 */
    int32_t small_search;       /* -1 or 1: one workgroup per pair where it fits, 0: never */
    int32_t level1_from_level0; /* -1: rule (sets of >= 96 Mi level-0 pixels), 0: never, 1: always */
    int32_t search_rows[16];    /* per level: 0, or a multiple of 4 in 4 .. 64 */
    int32_t search_lanes[16];   /* per level: 0, 8, 16, 32 or 64 */
    float step_ms;              /* tuners: median time of one call with this shape */
    float default_ms;           /* tuners: the same with the built-in shape */
} mtb_launch_shape;

/*
 * Tunes the launch shape of mtb_align_stack for these images: times whole
 * alignments (median of 7 after a warm-up, HIP events on `stream`) under the
 * built-in shape and under candidates changed one knob at a time (pyramid
 * 50/75/150/200 %, tile groups of 2 and 4, bitmaps 50/75 %, 2 and 8
 * wavefronts, the search by the launches above where one workgroup would
 * take the pair, and unless one workgroup searches: one coarse level fewer
 * or more, and at each fine level every
 * stream width and the rows halved or doubled), keeps a change only if it is
 * at least 2 % faster, stores the result in the table and writes it to
 * *h_out.  Arguments as for mtb_align_stack; d_shifts and d_errs receive the
 * results of the last call (identical under every shape).
 * Errors: as mtb_align_stack, MTB_ERR_INVALID_ARG for a null h_out.
 */
mtb_status mtb_tune_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width, int32_t height,
                          int64_t row_stride, int32_t levels, int32_t exclude_range, int32_t ref_index,
                          void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                          void *stream, mtb_launch_shape *h_out);

/* Stores *shape for the key (e.g. a shape tuned in an earlier run).
 * Errors: MTB_ERR_INVALID_ARG (null shape, a field out of range, invalid sizes). */
mtb_status mtb_set_shape(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels,
                         const mtb_launch_shape *shape);

/* The stored shape for the key into *h_out.
 * Errors: MTB_ERR_INVALID_ARG (null h_out, or no shape stored for the key). */
mtb_status mtb_tuned_shape(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels,
                           mtb_launch_shape *h_out);

/* Forgets every stored shape. */
void mtb_tune_reset(void);

/*
 * Writes every stored shape to the text file `path`, under a first line that
 * names the current device's architecture and the HIP runtime version.
 * Errors: MTB_ERR_INVALID_ARG (null path, file not writable),
 *         MTB_ERR_UNSUPPORTED (no device to name).
 */
mtb_status mtb_tune_save(const char *path);

/*
 * Stores the shapes of a file written by mtb_tune_save, if its first line
 * names the current device's architecture and HIP runtime version (shapes
 * tuned elsewhere are skipped whole: *h_loaded = 0); *h_loaded receives the
 * number stored.  The file is read completely before anything is stored.
 * Errors: MTB_ERR_INVALID_ARG (null pointer, unreadable or malformed file,
 *         a shape out of range), MTB_ERR_UNSUPPORTED (no device).
 */
mtb_status mtb_tune_load(const char *path, int32_t *h_loaded);

/*
 * For tests of error handling (callers that must survive a failed launch):
 * after `after` further kernel launches from the calling thread succeed, the
 * next one returns its failure without being issued, once, so the library
 * call that made it returns MTB_ERR_DEVICE; `after` < 0 cancels.  Nothing
 * faults on the device: the failing kernel is never launched.
 */
mtb_status mtb_test_fail_launch(int32_t after);

/*
 * For tests of the pyramid's histogram merge: the workgroup count of the last
 * k_pyramid launch made by the calling thread, and 1 if that launch merged
 * histograms through per-XCD copies (launches with many workgroups per
 * image), 0 if its workgroups added into the histograms directly.
 * Errors: MTB_ERR_INVALID_ARG (a null pointer, or no launch yet on this thread).
 */
mtb_status mtb_test_last_pyramid(int32_t *h_blocks, int32_t *h_merged);

/*
 * Translates every image of a stack by its shift (Section III-B: the shift
 * found for an exposure is applied to it, bringing it onto the reference):
 *   out_i[y][x] = in_i[y - dy_i][x - dx_i]   (all three channels)
 * Where (x - dx_i, y - dy_i) falls outside the image the paper says nothing;
 * `fill` chooses zeros (MTB_FILL_ZERO) or the nearest edge pixel
 * (MTB_FILL_EDGE, coordinates clamped into the image).
 *   h_d_rgb          host array of n device pointers, the input images (as for mtb_align_stack)
 *   d_shifts         device int32[n][2]: (dx, dy) per image, e.g. mtb_align_stack's d_shifts
 *   h_d_out          host array of n device pointers: height rows of out_stride bytes each;
 *                    bytes past 3 * width of a row are not written; must not overlap the inputs
 *   out_stride       >= 3 * width
 * Errors: MTB_ERR_INVALID_ARG (null pointers, sizes, strides, fill, n), MTB_ERR_DEVICE.
 */
#define MTB_FILL_ZERO 0
#define MTB_FILL_EDGE 1
mtb_status mtb_apply_shifts(const uint8_t *const *h_d_rgb, int32_t n, int32_t width, int32_t height,
                            int64_t row_stride, const int32_t *d_shifts, int32_t fill,
                            uint8_t *const *h_d_out, int64_t out_stride, void *stream);

/*
 * Host-staged input (Section II: every input image is copied to GPU memory
 * once; Section IV: that host-to-device transfer is part of the measured
 * time): enqueues on `stream` one 2-D copy of an RGB image from host memory
 * into device memory (3 * width bytes of each of `height` rows).  With h_rgb
 * in pinned memory (hipHostMalloc) the copy is an asynchronous DMA that
 * overlaps kernels on other streams; with pageable memory it may return only
 * once the copy is done.  The host buffer must stay valid until the copy has run.  Not a step
 * of the alignment: plumbing for callers whose frames arrive in host memory.
 * Speed: with h_rgb, d_rgb, both strides and 3 * width all multiples of 4 the
 * copy ran at 47-56 GB/s on MI355X over PCIe; a misaligned start address cut
 * that to about 6 GB/s and a row length that is not a multiple of 4 to under
 * 1 GB/s (row by row).  Callers staging crops can widen them to whole groups
 * of four pixels and align a view inside the copy.
 *   h_rgb, src_stride    host image, rows src_stride >= 3 * width bytes apart
 *   d_rgb, dst_stride    device destination, rows dst_stride >= 3 * width apart
 * Errors: MTB_ERR_INVALID_ARG (null pointers, sizes, strides), MTB_ERR_DEVICE.
 */
mtb_status mtb_stage_rgb(const uint8_t *h_rgb, int64_t src_stride, int32_t width, int32_t height,
                         uint8_t *d_rgb, int64_t dst_stride, void *stream);

/*
 * One item of a batch: a reference and a moving RGB image of the same size
 * and row stride (see Images above), aligned with `levels` levels.
 */
typedef struct mtb_batch_item {
    const uint8_t *d_ref_rgb;
    const uint8_t *d_mov_rgb;
    int64_t row_stride;
    int32_t width, height;
    int32_t levels;
    int32_t reserved; /* must be 0 */
} mtb_batch_item;

#define MTB_MAX_BATCH 4096 /* items per mtb_align_batch call */

/* Bytes of the workspace mtb_align_batch needs for these items (one range
 * per stream lane, each sized for the largest group); 0 if the item list or
 * any item is invalid. */
size_t mtb_batch_workspace_bytes(const mtb_batch_item *h_items, int32_t n_items);

/*
 * Many independent pairs of uneven sizes in one call: for every item, the
 * pairwise alignment of Section III-A (as mtb_align_pair on the items' own
 * pyramids and bitmaps, built as in mtb_build_pyramid and mtb_bitmaps).
 * Items of equal width, height, row stride and level count are processed
 * together, up to 16 pairs (32 images) per launch of each pass, with the
 * launch shape the table holds for the group's key.  The groups run on up to
 * four streams of the library (created once per host thread and device, at
 * default priority), forked from `stream` and joined back into it with
 * events, each lane with its own range of the workspace, so that one
 * group's latency-bound search overlaps another group's passes; work later
 * enqueued on `stream` follows the whole batch.  The call enqueues a
 * fixed sequence of kernels (no host synchronisation, no memset), so it can be
 * captured in a HIP graph and replayed.
 *   h_items          host array of n_items items (1 .. MTB_MAX_BATCH)
 *   exclude_range    as for mtb_bitmaps (Ward: 4)
 *   d_workspace      >= mtb_batch_workspace_bytes(h_items, n_items) bytes
 *   d_shifts         int32[n_items][2] receives (dx, dy) per item
 *   d_errs           uint32[n_items] receives each item's level-0 error
 * Errors: MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
mtb_status mtb_align_batch(const mtb_batch_item *h_items, int32_t n_items, int32_t exclude_range,
                           void *d_workspace, size_t workspace_bytes, int32_t *d_shifts,
                           uint32_t *d_errs, void *stream);

/* One exposure stack of a stacked batch (see mtb_align_batch_stacks). */
typedef struct mtb_batch_stack {
    const uint8_t *const *d_rgb; /* host array of n device RGB images, one size and row stride */
    int32_t n;                   /* images, 1 .. MTB_MAX_STACK */
    int32_t ref_index;           /* reference image, -1 for n / 2 */
    int64_t row_stride;
    int32_t width, height;
    int32_t levels;
    int32_t reserved;            /* must be 0 */
} mtb_batch_stack;

/* Bytes of the workspace mtb_align_batch_stacks needs; 0 if the item list
 * or any item is invalid. */
size_t mtb_batch_stacks_workspace_bytes(const mtb_batch_stack *h_items, int32_t n_items);

/*
 * Many exposure stacks of uneven sizes in one call: every stack aligned as
 * mtb_align_stack aligns it (Section III-A, III-B: each image against the
 * stack's reference, each image's pyramid and bitmaps built once).  Stacks
 * of equal width, height, row stride and level count share launch sets, up
 * to 32 images per launch of each pass (a stack is never split), which run
 * on the library's stream lanes as in mtb_align_batch, with the launch shape
 * the table holds for each set's key.  Output rows follow the items: the
 * rows of item k start after those of items 0 .. k-1, one per image; the
 * reference's row holds (0, 0) and error 0.  Every row is cleared on
 * `stream` before the lanes fork.
 *   h_items          host array of n_items stacks (1 .. MTB_MAX_BATCH)
 *   exclude_range    as for mtb_bitmaps (Ward: 4)
 *   d_workspace      >= mtb_batch_stacks_workspace_bytes(h_items, n_items) bytes
 *   d_shifts         int32[rows][2], rows = the items' images together
 *   d_errs           uint32[rows]
 * Errors: MTB_ERR_INVALID_ARG, MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
mtb_status mtb_align_batch_stacks(const mtb_batch_stack *h_items, int32_t n_items, int32_t exclude_range,
                                  void *d_workspace, size_t workspace_bytes, int32_t *d_shifts,
                                  uint32_t *d_errs, void *stream);

/*
 * Tunes the launch shapes of a batch: for each distinct group key (2 x pairs
 * of the group, width, height, levels, row-stride class; see the launch
 * shapes above), in order of first appearance, times the whole batch under
 * the candidate shapes of mtb_tune_stack for that key (the other keys at
 * their current shapes) and stores the winner in the table; *h_tuned
 * receives the number of keys tuned.  Arguments as for mtb_align_batch;
 * d_shifts and d_errs receive the results of a last call with the tuned
 * shapes (identical under every shape).
 * Errors: as mtb_align_batch, MTB_ERR_INVALID_ARG for a null h_tuned.
 */
mtb_status mtb_tune_batch(const mtb_batch_item *h_items, int32_t n_items, int32_t exclude_range,
                          void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                          void *stream, int32_t *h_tuned);

/*
 * Quadrant check for rotation (Section II: to find out whether a pair needs
 * rotational alignment, the image is split into quadrants and each quadrant is
 * aligned on its own).  The reference and moving images are cut into four
 * quadrants, q = 0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right,
 * split at column width / 2 and row height / 2, and each quadrant pair is
 * aligned as mtb_align_pair would align it (its own pyramids, medians and
 * bitmaps).  A rotation is flagged when two quadrants' shifts differ by more
 * than `tolerance` pixels along either axis (the paper gives no threshold).
 *   d_ref_rgb, d_mov_rgb  device RGB images (same size and stride)
 *   levels               1 .. mtb_max_levels(width / 2, height / 2)
 *   d_workspace          >= mtb_quadrant_workspace_bytes(width, height, row_stride, levels)
 *   d_shifts             int32[4][2] receives each quadrant's (dx, dy)
 *   d_errs               uint32[4] receives each quadrant's level-0 error
 *   d_flag               int32[1] receives 1 if a rotation is flagged, else 0
 * Errors: MTB_ERR_INVALID_ARG (pointers, sizes, stride, levels, tolerance < 0),
 *         MTB_ERR_WORKSPACE, MTB_ERR_DEVICE.
 */
size_t mtb_quadrant_workspace_bytes(int32_t width, int32_t height, int64_t row_stride, int32_t levels);
mtb_status mtb_align_quadrants(const uint8_t *d_ref_rgb, const uint8_t *d_mov_rgb, int32_t width,
                               int32_t height, int64_t row_stride, int32_t levels,
                               int32_t exclude_range, int32_t tolerance, void *d_workspace,
                               size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                               int32_t *d_flag, void *stream);

/*
 * Per-kernel timing for benchmarks.  Between mtb_profile_begin and
 * mtb_profile_end, every kernel that library calls made from the calling
 * thread launch is bracketed by two HIP events recorded on its stream; with
 * kernel_name non-NULL only kernels of that name are (names as listed by
 * rocprofv3, e.g. "k_pyramid").
 * mtb_profile_end waits for those events and writes one entry per kernel
 * name (launch count and summed event-to-event milliseconds) into h_out
 * (capacity entries), the number of entries into *h_count.
 * Errors: MTB_ERR_INVALID_ARG (begin while on / end while off / name of
 *         48 characters or more),
 *         MTB_ERR_WORKSPACE (more kernel names than capacity; the first
 *         capacity are still filled), MTB_ERR_DEVICE (an event failed).
 */
typedef struct mtb_kernel_time {
    char name[48];
    int64_t launches;
    double total_ms;
} mtb_kernel_time;

mtb_status mtb_profile_begin(const char *kernel_name);
mtb_status mtb_profile_end(mtb_kernel_time *h_out, int32_t capacity, int32_t *h_count);

/*
 * While profiling is on, mtb_profile_pause(1) stops bracketing new launches
 * and mtb_profile_pause(0) resumes; events already recorded are kept for
 * mtb_profile_end.  Nothing waits for the device.  Lets a benchmark time a
 * sample of its launches without the events' cost on every one.
 * Errors: MTB_ERR_INVALID_ARG when profiling is off.
 */
mtb_status mtb_profile_pause(int32_t paused);

/*
 * Measurement yardstick: one launch of a plain streaming kernel, so that a
 * benchmark can time the rate this device reaches for the passes' own mixes
 * of reads and writes (the pyramid pass reads 3 bytes per byte written, the
 * bitmaps pass 4).  With write_bytes > 0 it reads R = read_bytes /
 * write_bytes (integer part, 1 .. 4) contiguous 16-byte words of d_src per
 * 16-byte word it writes to d_dst (one nontemporal store), write_bytes / 16
 * times; with write_bytes = 0 it reads read_bytes of d_src in runs of four
 * words and writes nothing.  Both pointers 16-byte aligned; d_dst may be
 * NULL when write_bytes is 0.  The bytes written carry no meaning.
 * Errors: MTB_ERR_INVALID_ARG (null or misaligned pointers, less than one
 *         word, a ratio outside 1 .. 4), MTB_ERR_UNSUPPORTED (no device),
 *         MTB_ERR_DEVICE.
 */
mtb_status mtb_probe_stream(const void *d_src, size_t read_bytes, void *d_dst, size_t write_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MTB_H */
