// mtb_api.hip -- the C-ABI entry points of libmtb: argument validation, buffer
// layout, and the launch sequence of each call.  No device memory is
// allocated here; every buffer comes from the caller.

#include <mutex>
#include <string.h>

#include "mtb_internal.h"

namespace mtb {

int32_t max_levels(int32_t W, int32_t H)
{
    if (W < 1 || H < 1)
        return 0;
    int32_t L = 0;
    while (L < 31 && (W >> L) >= 1 && (H >> L) >= 1)
        ++L;
    return L;
}

bool make_geometry(int32_t W, int32_t H, int32_t L, Geometry *g)
{
    if (W < 1 || H < 1 || (int64_t)W * H >= ((int64_t)1 << 31))
        return false;
    if (L < 1 || L > max_levels(W, H) || L > kMaxLevels)
        return false;
    memset(g, 0, sizeof(*g));
    g->W = W;
    g->H = H;
    g->L = L;
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        LevelGeom &lv = g->lv[l];
        lv.w = W >> l;
        lv.h = H >> l;
        // Rows padded to 128 pixels: gray rows start on 128-byte lines.
        lv.wpr = 2 * ((lv.w + 127) / 128);
        lv.gray_pitch = 64 * (int64_t)lv.wpr;
        lv.gray_off = off;
        off = align_up(off + lv.gray_pitch * lv.h, kAlign);
    }
    g->hist_off = off;
    off = align_up(off + (int64_t)L * 256 * 4, kAlign);
    g->pyramid_bytes = off;
    // The search reads up to two words either side of a bitmap row (and masks
    // them out): a leading guard keeps those reads inside the buffer before
    // the first plane; the medians follow the last plane.
    off = kAlign;
    for (int l = 0; l < L; ++l) {
        LevelGeom &lv = g->lv[l];
        const int64_t plane = 8 * (int64_t)lv.wpr * lv.h;
        lv.tb_off = off;
        off = align_up(off + plane, kAlign);
        lv.eb_off = off;
        off = align_up(off + plane, kAlign);
    }
    g->med_off = off;
    off = align_up(off + (int64_t)L * 4, kAlign);
    g->bitmaps_bytes = off;
    return true;
}

namespace {

// Words of search state per pair, padded to 256 bytes.
int64_t state_stride_words(int32_t L) { return align_up(pair_state_words(L), kAlign / 4); }

struct DeviceInfo {
    int cus = 0;
    bool ok = false;
    bool known = false;
};

std::mutex g_dev_mutex;
DeviceInfo g_dev[64];

// Compute-unit count of the current device, or 0 if it is not a usable gfx950.
int current_device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceInfo &d = g_dev[dev];
    if (!d.known) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return 0;
        d.known = true;
        d.ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        d.cus = prop.multiProcessorCount;
    }
    return d.ok ? d.cus : 0;
}

mtb_status device_status(hipError_t e) { return e == hipSuccess ? MTB_OK : MTB_ERR_DEVICE; }

// Alignment (16, 4 or 1 bytes) that every row start of an image has.
int row_alignment(const uint8_t *p, int64_t stride)
{
    const uintptr_t v = (uintptr_t)p | (uintptr_t)stride;
    return v % 16 == 0 ? 16 : (v % 4 == 0 ? 4 : 1);
}

void fill_chunk_starts(const Geometry &g, int64_t *cs)
{
    cs[0] = 0;
    for (int l = 0; l < g.L; ++l) {
        const int64_t words = (int64_t)g.lv[l].h * g.lv[l].wpr;
        cs[l + 1] = cs[l] + (words + kChunkWords - 1) / kChunkWords;
    }
}

}  // namespace
}  // namespace mtb

using namespace mtb;

extern "C" {

const char *mtb_status_string(mtb_status status)
{
    switch (status) {
    case MTB_OK:
        return "MTB_OK";
    case MTB_ERR_INVALID_ARG:
        return "MTB_ERR_INVALID_ARG";
    case MTB_ERR_WORKSPACE:
        return "MTB_ERR_WORKSPACE";
    case MTB_ERR_DEVICE:
        return "MTB_ERR_DEVICE";
    case MTB_ERR_UNSUPPORTED:
        return "MTB_ERR_UNSUPPORTED";
    }
    return "MTB_ERR_UNKNOWN";
}

int32_t mtb_max_levels(int32_t width, int32_t height)
{
    const int32_t L = max_levels(width, height);
    return L > kMaxLevels ? kMaxLevels : L;
}

mtb_status mtb_get_layout(int32_t width, int32_t height, int32_t levels, mtb_layout *out)
{
    Geometry g;
    if (!out || !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    out->width = width;
    out->height = height;
    out->levels = levels;
    for (int l = 0; l < levels; ++l) {
        out->level_width[l] = g.lv[l].w;
        out->level_height[l] = g.lv[l].h;
        out->words_per_row[l] = g.lv[l].wpr;
        out->gray_offset[l] = g.lv[l].gray_off;
        out->gray_pitch[l] = g.lv[l].gray_pitch;
        out->tb_offset[l] = g.lv[l].tb_off;
        out->eb_offset[l] = g.lv[l].eb_off;
    }
    out->hist_offset = g.hist_off;
    out->pyramid_bytes = g.pyramid_bytes;
    out->median_offset = g.med_off;
    out->bitmaps_bytes = g.bitmaps_bytes;
    return MTB_OK;
}

size_t mtb_pyramid_bytes(int32_t width, int32_t height, int32_t levels)
{
    Geometry g;
    return make_geometry(width, height, levels, &g) ? (size_t)g.pyramid_bytes : 0;
}

size_t mtb_bitmaps_bytes(int32_t width, int32_t height, int32_t levels)
{
    Geometry g;
    return make_geometry(width, height, levels, &g) ? (size_t)g.bitmaps_bytes : 0;
}

size_t mtb_pair_workspace_bytes(int32_t levels)
{
    if (levels < 1 || levels > kMaxLevels)
        return 0;
    return (size_t)(state_stride_words(levels) + align_up(kTicketWords, kAlign / 4)) * 4;  // state, tickets
}

size_t mtb_stack_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t levels)
{
    Geometry g;
    if (n < 1 || n > kMaxStack || !make_geometry(width, height, levels, &g))
        return 0;
    // pyramids, bitmaps, search state, ticket counters, plus slack to align the start
    return (size_t)(n * (g.pyramid_bytes + g.bitmaps_bytes) + (n - 1) * state_stride_words(levels) * 4 +
                    align_up(4 * kTicketWords, kAlign) + kAlign);
}

mtb_status mtb_build_pyramid(const uint8_t *d_rgb, int32_t width, int32_t height,
                             int64_t row_stride, int32_t levels, void *d_pyramid,
                             size_t pyramid_bytes, void *stream)
{
    Geometry g;
    if (!d_rgb || !d_pyramid || !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    if (row_stride < 3 * (int64_t)width)
        return MTB_ERR_INVALID_ARG;
    if (pyramid_bytes < (size_t)g.pyramid_bytes)
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *pyr = (uint8_t *)d_pyramid;

    ZeroArgs z;
    memset(&z, 0, sizeof(z));
    z.ptr[0] = (uint32_t *)(pyr + g.hist_off);
    z.words[0] = (int64_t)levels * 256;
    z.count = 1;
    hipError_t e = launch_zero(z, s);
    if (e != hipSuccess)
        return MTB_ERR_DEVICE;

    PyramidArgs a;
    memset(&a, 0, sizeof(a));
    a.rgb[0] = d_rgb;
    a.pyr[0] = pyr;
    a.stride = row_stride;
    a.n = 1;
    a.align = row_alignment(d_rgb, row_stride);
    a.g = g;
    return device_status(launch_pyramid(a, cus, s));
}

mtb_status mtb_bitmaps(const void *d_pyramid, int32_t width, int32_t height, int32_t levels,
                       int32_t exclude_range, void *d_bitmaps, size_t bitmaps_bytes, void *stream)
{
    Geometry g;
    if (!d_pyramid || !d_bitmaps || !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    if (exclude_range < 0 || exclude_range > 255)
        return MTB_ERR_INVALID_ARG;
    if (bitmaps_bytes < (size_t)g.bitmaps_bytes)
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    BitmapArgs a;
    memset(&a, 0, sizeof(a));
    a.pyr[0] = (const uint8_t *)d_pyramid;
    a.bm[0] = (uint8_t *)d_bitmaps;
    a.n = 1;
    a.exclude = exclude_range;
    a.g = g;
    fill_chunk_starts(g, a.chunk_start);
    return device_status(launch_bitmaps(a, cus, (hipStream_t)stream));
}

mtb_status mtb_align_pair(const void *d_bm_ref, const void *d_bm_mov, int32_t width,
                          int32_t height, int32_t levels, void *d_workspace,
                          size_t workspace_bytes, int32_t *d_shift, uint32_t *d_err,
                          uint32_t *d_trace, int32_t *d_level_shifts, void *stream)
{
    Geometry g;
    if (!d_bm_ref || !d_bm_mov || !d_workspace || !d_shift || !d_err ||
        !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    if (workspace_bytes < mtb_pair_workspace_bytes(levels))
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *state = (uint32_t *)d_workspace;

    ZeroArgs z;
    memset(&z, 0, sizeof(z));
    z.ptr[0] = state;
    z.words[0] = state_stride_words(levels) + kTicketWords;  // counters, bases, surfaces, tickets
    z.count = 1;
    if (launch_zero(z, s) != hipSuccess)
        return MTB_ERR_DEVICE;

    SearchArgs a;
    memset(&a, 0, sizeof(a));
    a.ref[0] = (const uint8_t *)d_bm_ref;
    a.mov[0] = (const uint8_t *)d_bm_mov;
    a.state = state;
    a.done = state + state_stride_words(levels);
    a.state_stride = state_stride_words(levels);
    a.npairs = 1;
    a.out.pair_image[0] = 0;
    a.out.n_out = 1;
    a.out.shifts = d_shift;
    a.out.errs = d_err;
    a.out.trace = d_trace;
    a.out.level_shifts = d_level_shifts;
    a.g = g;
    return device_status(launch_search(a, cus, s));
}

mtb_status mtb_align_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                           int32_t height, int64_t row_stride, int32_t levels,
                           int32_t exclude_range, int32_t ref_index, void *d_workspace,
                           size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                           uint32_t *d_trace, void *stream)
{
    Geometry g;
    if (!h_d_rgb || n < 1 || n > kMaxStack || !d_workspace || !d_shifts || !d_errs ||
        !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    if (row_stride < 3 * (int64_t)width || exclude_range < 0 || exclude_range > 255)
        return MTB_ERR_INVALID_ARG;
    const int ref = ref_index < 0 ? n / 2 : ref_index;
    if (ref >= n)
        return MTB_ERR_INVALID_ARG;
    int align = 16;
    for (int i = 0; i < n; ++i) {
        if (!h_d_rgb[i])
            return MTB_ERR_INVALID_ARG;
        const int ai = row_alignment(h_d_rgb[i], row_stride);
        align = ai < align ? ai : align;
    }
    if (workspace_bytes < mtb_stack_workspace_bytes(n, width, height, levels))
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;

    // Workspace: pyramids, bitmaps, then search state, from a 256-byte aligned start.
    uint8_t *base = (uint8_t *)align_up((int64_t)(uintptr_t)d_workspace, kAlign);
    uint8_t *pyr0 = base;
    uint8_t *bm0 = pyr0 + n * g.pyramid_bytes;
    uint32_t *state = (uint32_t *)(bm0 + n * g.bitmaps_bytes);
    const int64_t sstride = state_stride_words(levels);
    const int npairs = n - 1;
    uint32_t *done = state + sstride * npairs;

    ZeroArgs z;
    memset(&z, 0, sizeof(z));
    for (int i = 0; i < n; ++i) {
        z.ptr[i] = (uint32_t *)(pyr0 + i * g.pyramid_bytes + g.hist_off);
        z.words[i] = (int64_t)levels * 256;
    }
    z.ptr[n] = state;
    z.words[n] = sstride * npairs + kTicketWords;  // every pair's search state, then the tickets
    z.count = n + 1;
    // The reference's output rows stay zero; the search writes every other row.
    z.ptr[z.count] = (uint32_t *)d_shifts;
    z.words[z.count++] = 2 * (int64_t)n;
    z.ptr[z.count] = d_errs;
    z.words[z.count++] = n;
    if (d_trace) {
        z.ptr[z.count] = d_trace;
        z.words[z.count++] = 9 * (int64_t)levels * n;
    }
    if (launch_zero(z, s) != hipSuccess)
        return MTB_ERR_DEVICE;

    PyramidArgs pa;
    memset(&pa, 0, sizeof(pa));
    for (int i = 0; i < n; ++i) {
        pa.rgb[i] = h_d_rgb[i];
        pa.pyr[i] = pyr0 + i * g.pyramid_bytes;
    }
    pa.stride = row_stride;
    pa.n = n;
    pa.align = align;
    pa.g = g;
    if (launch_pyramid(pa, cus, s) != hipSuccess)
        return MTB_ERR_DEVICE;

    BitmapArgs ba;
    memset(&ba, 0, sizeof(ba));
    for (int i = 0; i < n; ++i) {
        ba.pyr[i] = pyr0 + i * g.pyramid_bytes;
        ba.bm[i] = bm0 + i * g.bitmaps_bytes;
    }
    ba.n = n;
    ba.exclude = exclude_range;
    ba.g = g;
    fill_chunk_starts(g, ba.chunk_start);
    if (launch_bitmaps(ba, cus, s) != hipSuccess)
        return MTB_ERR_DEVICE;
    if (npairs == 0)
        return MTB_OK;

    SearchArgs sa;
    memset(&sa, 0, sizeof(sa));
    int p = 0;
    for (int i = 0; i < n; ++i) {
        if (i == ref)
            continue;
        sa.ref[p] = bm0 + ref * g.bitmaps_bytes;
        sa.mov[p] = bm0 + i * g.bitmaps_bytes;
        sa.out.pair_image[p] = i;
        ++p;
    }
    sa.state = state;
    sa.done = done;
    sa.state_stride = sstride;
    sa.npairs = npairs;
    sa.out.n_out = n;
    sa.out.shifts = d_shifts;
    sa.out.errs = d_errs;
    sa.out.trace = d_trace;
    sa.out.level_shifts = nullptr;
    sa.g = g;
    return device_status(launch_search(sa, cus, s));
}

}  // extern "C"
