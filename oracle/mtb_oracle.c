/*
 * mtb_oracle.c -- CPU oracle for Median Threshold Bitmap (MTB) translational
 * alignment.  TEST INFRASTRUCTURE ONLY: the parity tests, the smoke check and
 * the CPU-baseline leg of the benchmark call it; the product path never does.
 *
 * Plain, slow, obviously correct C: one byte per pixel for every image and
 * bitmap, no bit packing, no tiling, no fusion, single-threaded.  Each
 * function cites the passage of the paper (Alpay, Aydemir, Akyuz,
 * "Accelerating Translational Image Registration for HDR Images on GPU",
 * arXiv 2007.06483) that it follows.  Where the paper is silent the reading
 * used is stated at the function.
 *
 * Conventions shared by all functions:
 *   - an RGB image is H rows of W interleaved R,G,B bytes, rows `stride` bytes apart;
 *   - a gray image or bitmap of level l is W_l x H_l bytes, packed (pitch W_l),
 *     W_l = W >> l, H_l = H >> l;
 *   - a "pyramid" array holds levels 0..L-1 back to back, level l starting at
 *     oracle_level_offset(W, H, l).
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

/* Offset of level l inside a back-to-back pyramid array of bytes. */
int64_t oracle_level_offset(int32_t width, int32_t height, int32_t level)
{
    int64_t off = 0;
    for (int32_t l = 0; l < level; ++l)
        off += (int64_t)(width >> l) * (int64_t)(height >> l);
    return off;
}

/*
 * Gray-scale conversion (Section III-A: exposures are first turned into gray
 * scale).  The paper gives no weights; Ward's integer weights are used:
 * g = (54 R + 183 G + 19 B) >> 8.  The weights sum to 256, so g <= 255.
 */
void oracle_gray(const uint8_t *rgb, int32_t width, int32_t height, int64_t stride,
                 uint8_t *gray)
{
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            const uint8_t *p = rgb + (int64_t)y * stride + 3 * (int64_t)x;
            uint32_t r = p[0], g = p[1], b = p[2];
            gray[(int64_t)y * width + x] = (uint8_t)((54u * r + 183u * g + 19u * b) >> 8);
        }
    }
}

/*
 * One pyramid step (Section III-A: the gray images are downsampled by halving
 * both dimensions; Fig. 2).  Reading: each output pixel is the floor of the
 * mean of the 2x2 block above it; an odd last row or column of the input is
 * dropped.  out is (win >> 1) x (hin >> 1).
 */
void oracle_downsample(const uint8_t *in, int32_t win, int32_t hin, uint8_t *out)
{
    int32_t wo = win >> 1, ho = hin >> 1;
    for (int32_t y = 0; y < ho; ++y) {
        for (int32_t x = 0; x < wo; ++x) {
            uint32_t s = (uint32_t)in[(int64_t)(2 * y) * win + 2 * x]
                       + (uint32_t)in[(int64_t)(2 * y) * win + 2 * x + 1]
                       + (uint32_t)in[(int64_t)(2 * y + 1) * win + 2 * x]
                       + (uint32_t)in[(int64_t)(2 * y + 1) * win + 2 * x + 1];
            out[(int64_t)y * wo + x] = (uint8_t)(s >> 2);
        }
    }
}

/* 256-bin histogram of one gray image (Section III-B, per pyramid level). */
void oracle_histogram(const uint8_t *gray, int64_t npix, uint32_t *hist)
{
    for (int v = 0; v < 256; ++v)
        hist[v] = 0;
    for (int64_t i = 0; i < npix; ++i)
        hist[gray[i]] += 1;
}

/*
 * Median from the histogram (Sections III-A and III-B).  For an even count
 * the paper is silent; the lower median is used: the smallest value v whose
 * cumulative count reaches ceil(npix / 2), i.e. element (npix - 1) / 2 of the
 * sorted pixels.  Returns 0 for an empty image.
 */
int32_t oracle_median(const uint32_t *hist, int64_t npix)
{
    int64_t need = (npix + 1) / 2, cum = 0;
    for (int v = 0; v < 256; ++v) {
        cum += hist[v];
        if (cum >= need && need > 0)
            return v;
    }
    return 0;
}

/*
 * Threshold and exclusion bitmaps, one byte (0 or 1) per pixel.
 * Threshold (Section III-A): pixels at or below the median map to 0, the
 * others to 1:  T = [g > m].
 * Exclusion (Section III-B): the text's polarity would keep only the noisy
 * pixels, contradicting its stated purpose of removing them; the reading
 * used keeps the pixels away from the median:  E = [|g - m| > x], x = 4.
 */
void oracle_bitmaps(const uint8_t *gray, int64_t npix, int32_t median, int32_t exclude,
                    uint8_t *tb, uint8_t *eb)
{
    for (int64_t i = 0; i < npix; ++i) {
        int32_t g = gray[i];
        int32_t d = g - median;
        if (d < 0)
            d = -d;
        tb[i] = (uint8_t)(g > median);
        eb[i] = (uint8_t)(d > exclude);
    }
}

/*
 * Error of one candidate shift c = (cx, cy) at one level (Sections III-A and
 * III-B): the shifted moving bitmaps are XORed with the reference threshold
 * bitmap, both exclusion bitmaps are ANDed on, and the set pixels counted
 * over the reference frame.  The shift moves the moving image's content:
 * (S_c B)[y][x] = B[y - cy][x - cx], and a pixel shifted in from outside the
 * image is 0 in both of its bitmaps (reading: zero fill; the paper is silent).
 */
int64_t oracle_shift_error(const uint8_t *tr, const uint8_t *er, const uint8_t *tm,
                           const uint8_t *em, int32_t w, int32_t h, int32_t cx, int32_t cy)
{
    int64_t count = 0;
    for (int32_t y = 0; y < h; ++y) {
        for (int32_t x = 0; x < w; ++x) {
            int32_t sy = y - cy, sx = x - cx;
            uint8_t t = 0, e = 0;
            if (sy >= 0 && sy < h && sx >= 0 && sx < w) {
                t = tm[(int64_t)sy * w + sx];
                e = em[(int64_t)sy * w + sx];
            }
            int64_t i = (int64_t)y * w + x;
            count += (uint8_t)((tr[i] ^ t) & er[i] & e);
        }
    }
    return count;
}

/*
 * Gray pyramid with histograms and medians for one RGB image (Sections
 * III-A and III-B).  gray_pyr receives levels 0..L-1 back to back,
 * hist is [L][256], median is [L].
 */
void oracle_pyramid(const uint8_t *rgb, int32_t width, int32_t height, int64_t stride,
                    int32_t levels, uint8_t *gray_pyr, uint32_t *hist, int32_t *median)
{
    oracle_gray(rgb, width, height, stride, gray_pyr);
    for (int32_t l = 1; l < levels; ++l)
        oracle_downsample(gray_pyr + oracle_level_offset(width, height, l - 1),
                          width >> (l - 1), height >> (l - 1),
                          gray_pyr + oracle_level_offset(width, height, l));
    for (int32_t l = 0; l < levels; ++l) {
        int64_t np = (int64_t)(width >> l) * (int64_t)(height >> l);
        oracle_histogram(gray_pyr + oracle_level_offset(width, height, l), np, hist + 256 * l);
        median[l] = oracle_median(hist + 256 * l, np);
    }
}

/* Threshold and exclusion bitmaps of every level of a pyramid (same back-to-back layout). */
void oracle_pyramid_bitmaps(const uint8_t *gray_pyr, int32_t width, int32_t height,
                            int32_t levels, const int32_t *median, int32_t exclude,
                            uint8_t *tb_pyr, uint8_t *eb_pyr)
{
    for (int32_t l = 0; l < levels; ++l) {
        int64_t off = oracle_level_offset(width, height, l);
        int64_t np = (int64_t)(width >> l) * (int64_t)(height >> l);
        oracle_bitmaps(gray_pyr + off, np, median[l], exclude, tb_pyr + off, eb_pyr + off);
    }
}

/*
 * Coarse-to-fine search (Section III-A, Fig. 2; Section III-B).  Starting at
 * the coarsest level with offset (0, 0), the nine shifts within +-1 pixel of
 * the current offset are tested; the best becomes the level's shift, and the
 * offset is doubled before moving to the next finer level.  Nine tests per
 * level: 54 for six levels.
 * Tie-break (the paper is silent): candidates are visited dy-major
 * (dy = -1, 0, 1 outer; dx = -1, 0, 1 inner) and only a strictly smaller
 * error replaces the best, so the lowest (dy, dx) wins a tie.
 *
 * Outputs: shift[2] = (dx, dy) at level 0, *err = its level-0 error,
 * trace[L][9] (may be NULL) = error of candidate (dy+1)*3 + (dx+1) at each
 * level, level_shift[L][2] (may be NULL) = the shift chosen at each level.
 */
void oracle_search(const uint8_t *tr_pyr, const uint8_t *er_pyr, const uint8_t *tm_pyr,
                   const uint8_t *em_pyr, int32_t width, int32_t height, int32_t levels,
                   int32_t *shift, int64_t *err, int64_t *trace, int32_t *level_shift)
{
    int32_t bx = 0, by = 0, sx = 0, sy = 0;
    int64_t best = 0;
    for (int32_t l = levels - 1; l >= 0; --l) {
        int64_t off = oracle_level_offset(width, height, l);
        int32_t w = width >> l, h = height >> l;
        best = INT64_MAX;
        for (int32_t dy = -1; dy <= 1; ++dy) {
            for (int32_t dx = -1; dx <= 1; ++dx) {
                int64_t e = oracle_shift_error(tr_pyr + off, er_pyr + off, tm_pyr + off,
                                               em_pyr + off, w, h, bx + dx, by + dy);
                if (trace)
                    trace[9 * l + 3 * (dy + 1) + (dx + 1)] = e;
                if (e < best) {
                    best = e;
                    sx = bx + dx;
                    sy = by + dy;
                }
            }
        }
        if (level_shift) {
            level_shift[2 * l] = sx;
            level_shift[2 * l + 1] = sy;
        }
        bx = 2 * sx;
        by = 2 * sy;
    }
    shift[0] = sx;
    shift[1] = sy;
    *err = best;
}

/*
 * Pairwise alignment of two RGB images of the same size, end to end:
 * pyramid, histograms, medians and bitmaps of both, then the search.
 * Scratch memory is allocated here and freed before returning; returns 0 on
 * success and -1 if an allocation fails.
 */
int32_t oracle_align_pair(const uint8_t *rgb_ref, const uint8_t *rgb_mov, int32_t width,
                          int32_t height, int64_t stride, int32_t levels, int32_t exclude,
                          int32_t *shift, int64_t *err, int64_t *trace, int32_t *level_shift)
{
    int64_t total = oracle_level_offset(width, height, levels);
    uint8_t *buf = (uint8_t *)malloc((size_t)(6 * total));
    uint32_t *hist = (uint32_t *)malloc(sizeof(uint32_t) * 256 * (size_t)levels);
    int32_t *med = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)levels);
    if (!buf || !hist || !med) {
        free(buf);
        free(hist);
        free(med);
        return -1;
    }
    uint8_t *g_ref = buf, *g_mov = buf + total;
    uint8_t *tr = buf + 2 * total, *er = buf + 3 * total;
    uint8_t *tm = buf + 4 * total, *em = buf + 5 * total;
    oracle_pyramid(rgb_ref, width, height, stride, levels, g_ref, hist, med);
    oracle_pyramid(rgb_mov, width, height, stride, levels, g_mov, hist, med + levels);
    oracle_pyramid_bitmaps(g_ref, width, height, levels, med, exclude, tr, er);
    oracle_pyramid_bitmaps(g_mov, width, height, levels, med + levels, exclude, tm, em);
    oracle_search(tr, er, tm, em, width, height, levels, shift, err, trace, level_shift);
    free(buf);
    free(hist);
    free(med);
    return 0;
}

/*
 * Applying the found shift to a moving image (Section III-B: once the shift is
 * known the image is translated by it; Section III-A: the shift moves the
 * moving image onto the reference).  out[y][x] = in[y - dy][x - dx] for every
 * channel; where (x - dx, y - dy) falls outside the image the paper says
 * nothing, and two readings are offered: fill 0 writes zero bytes, fill 1
 * repeats the nearest edge pixel (coordinates clamped into the image).
 * Output rows are out_stride bytes apart; bytes past 3 * width are untouched.
 */
void oracle_apply_shift(const uint8_t *in, int32_t width, int32_t height, int64_t stride,
                        int32_t dx, int32_t dy, int32_t fill, uint8_t *out, int64_t out_stride)
{
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            int64_t sx = (int64_t)x - dx, sy = (int64_t)y - dy;
            const int inside = sx >= 0 && sx < width && sy >= 0 && sy < height;
            for (int c = 0; c < 3; ++c) {
                uint8_t v = 0;
                if (inside) {
                    v = in[sy * stride + 3 * sx + c];
                } else if (fill == 1) {
                    const int64_t cx = sx < 0 ? 0 : (sx >= width ? width - 1 : sx);
                    const int64_t cy = sy < 0 ? 0 : (sy >= height ? height - 1 : sy);
                    v = in[cy * stride + 3 * cx + c];
                }
                out[(int64_t)y * out_stride + 3 * (int64_t)x + c] = v;
            }
        }
    }
}
