// mtb_api.hip -- the C-ABI entry points of libmtb: argument validation, buffer
// layout, and the launch sequence of each call.  No device memory is
// allocated here; every buffer comes from the caller.

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdio.h>
#include <string.h>
#include <string>
#include <vector>

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
    g->hmerge_off = off;
    off = align_up(off + 4 * kHMergeWords, kAlign);
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
    // Byte maps (the paper's 255/0 representation, for comparison): the same
    // guard, a T and an E plane of gray_pitch-byte rows per level, medians.
    off = kAlign;
    for (int l = 0; l < L; ++l) {
        LevelGeom &lv = g->lv[l];
        const int64_t plane = lv.gray_pitch * lv.h;
        lv.bt_off = off;
        off = align_up(off + plane, kAlign);
        lv.be_off = off;
        off = align_up(off + plane, kAlign);
    }
    g->bmed_off = off;
    g->bytemaps_bytes = align_up(off + (int64_t)L * 4, kAlign);
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

// Launches of this thread still to succeed before an injected failure; -1: none.
thread_local int t_fail_after = -1;
// Workgroups and merge mode of this thread's last k_pyramid launch; -1: none yet.
thread_local int t_pyr_blocks = -1, t_pyr_merged = 0;

// Alignment (16, 4 or 1 bytes) that every row start of an image has.
int row_alignment(const uint8_t *p, int64_t stride)
{
    const uintptr_t v = (uintptr_t)p | (uintptr_t)stride;
    return v % 16 == 0 ? 16 : (v % 4 == 0 ? 4 : 1);
}

// First chunk of each level within one image.  With `pairs`, level 0 counts
// units of two rows by kPairWords words and level 1 none (its bitmaps come
// from level 0's units).
void fill_chunk_starts(const Geometry &g, int64_t *cs, bool pairs = false)
{
    cs[0] = 0;
    for (int l = 0; l < g.L; ++l) {
        const int64_t words = (int64_t)g.lv[l].h * g.lv[l].wpr;
        int64_t chunks = (words + kChunkWords - 1) / kChunkWords;
        if (pairs && l == 0)
            chunks = (int64_t)((g.lv[0].h + 1) / 2) * ((g.lv[0].wpr + kPairWords - 1) / kPairWords);
        else if (pairs && l == 1)
            chunks = 0;
        cs[l + 1] = cs[l] + chunks;
    }
}

// One launch set: n images of one size, each image's pyramid and bitmaps
// built once, then the search of npairs pairs of them (reference ref_img[p]
// against moving image mov_img[p], results in output row out_row[p]).
struct PairSet {
    const uint8_t *rgb[kMaxStack];
    int n = 0;
    int ref_img[kMaxStack], mov_img[kMaxStack], out_row[kMaxStack];
    int npairs = 0;
};

// Workspace bytes of a launch set (from a 256-byte aligned start): pyramids,
// bitmaps, each pair's search state, ticket counters.
int64_t set_workspace_bytes(const Geometry &g, int n, int npairs, bool bytemaps = false)
{
    return n * (g.pyramid_bytes + (bytemaps ? g.bytemaps_bytes : g.bitmaps_bytes)) +
           npairs * state_stride_words(g.L) * 4 + align_up(4 * kTicketWords, kAlign);
}

// Launch sets of at least this many level-0 pixels (n * W * H) form level 1's
// bitmaps from level 0's gray by default: below it the bitmaps pass's second
// median per wavefront costs more than the level-1 traffic it saves
// (measured: 2 x 6000x4000 +1.3 us, 4 x 4096x3072 +1.5 us, 3 x 6000x4000
// even, 5 x 6000x4000 -2.5 us, 7 x 6000x4000 -8 to -11 us).
constexpr int64_t kL1MinPixels = (int64_t)96 << 20;

// Whether a launch set of n images takes level 1's bitmaps from level 0's
// gray (and leaves level 1's gray unstored) under launch shape t.
bool level1_from_level0(const Geometry &g, int n, const LaunchTune &t)
{
    if (g.L < 2)
        return false;
    if (t.l1 >= 0)
        return t.l1 == 1;
    return (int64_t)n * g.W * g.H >= kL1MinPixels;
}

// Enqueues a launch set on s.  `ws` is 256-byte aligned; `zero` lists output
// regions to clear first (taken by value, its free slots are used here).
hipError_t enqueue_set(const PairSet &ps, const Geometry &g, int64_t stride, int align, int exclude,
                       uint8_t *ws, SearchOutputs out, ZeroArgs zero, int cus, hipStream_t s,
                       bool bytemaps = false, const LaunchTune &t = LaunchTune())
{
    const int n = ps.n, npairs = ps.npairs;
    const int64_t mb = bytemaps ? g.bytemaps_bytes : g.bitmaps_bytes;  // maps buffer per image
    // The packed bitmaps may take levels 0 and 1 from level 0's gray, and
    // level 1's gray is then not stored; the byte maps read every level's gray.
    const bool pairs = !bytemaps && level1_from_level0(g, n, t);
    uint8_t *pyr0 = ws;
    uint8_t *bm0 = pyr0 + n * g.pyramid_bytes;
    uint32_t *state = (uint32_t *)(bm0 + n * mb);
    const int64_t sstride = state_stride_words(g.L);

    for (int i = 0; i < n; ++i) {
        zero.ptr[zero.count] = (uint32_t *)(pyr0 + i * g.pyramid_bytes + g.hist_off);
        zero.words[zero.count++] = (g.pyramid_bytes - g.hist_off) / 4;  // histograms and merge scratch
    }
    zero.ptr[zero.count] = state;
    zero.words[zero.count++] = sstride * npairs + kTicketWords;  // every pair's search state, then the tickets
    hipError_t e = launch_zero(zero, s);
    if (e != hipSuccess)
        return e;

    PyramidArgs pa;
    memset(&pa, 0, sizeof(pa));
    for (int i = 0; i < n; ++i) {
        pa.rgb[i] = ps.rgb[i];
        pa.pyr[i] = pyr0 + i * g.pyramid_bytes;
    }
    pa.stride = stride;
    pa.n = n;
    pa.align = align;
    pa.skip_l1 = pairs;
    pa.g = g;
    e = launch_pyramid(pa, cus, s, t.pyr_pct, t.pyr_group_log2);
    if (e != hipSuccess)
        return e;

    BitmapArgs ba;
    memset(&ba, 0, sizeof(ba));
    for (int i = 0; i < n; ++i) {
        ba.pyr[i] = pyr0 + i * g.pyramid_bytes;
        ba.bm[i] = bm0 + i * mb;
    }
    ba.n = n;
    ba.exclude = exclude;
    ba.pairs = pairs;
    ba.g = g;
    fill_chunk_starts(g, ba.chunk_start, pairs);
    e = bytemaps ? launch_bytemaps(ba, cus, s) : launch_bitmaps(ba, cus, s, t.bm_pct, t.bm_waves);
    if (e != hipSuccess || npairs == 0)
        return e;

    SearchArgs sa;
    memset(&sa, 0, sizeof(sa));
    for (int p = 0; p < npairs; ++p) {
        sa.ref[p] = bm0 + ps.ref_img[p] * mb;
        sa.mov[p] = bm0 + ps.mov_img[p] * mb;
        out.pair_image[p] = ps.out_row[p];
    }
    sa.state = state;
    sa.done = state + sstride * npairs;
    sa.state_stride = sstride;
    sa.npairs = npairs;
    sa.out = out;
    sa.g = g;
    return bytemaps ? launch_search_bytes(sa, cus, s) : launch_search(sa, cus, s, &t);
}

// Tuned launch shapes, per (images, size, levels, row alignment); filled by
// mtb_tune_stack, mtb_tune_batch, mtb_set_shape and mtb_tune_load, read by the
// stack and batch calls.  A shape also serves, until one of their own is
// stored, the sizes of its bucket: same images, levels and row alignment, and
// a pixel count in the same half octave.
struct TuneKey {
    int n, w, h, levels, align;
    bool operator<(const TuneKey &o) const
    {
        return n != o.n ? n < o.n : w != o.w ? w < o.w : h != o.h ? h < o.h : levels != o.levels ? levels < o.levels
                                                                                                  : align < o.align;
    }
    bool operator==(const TuneKey &o) const
    {
        return n == o.n && w == o.w && h == o.h && levels == o.levels && align == o.align;
    }
};
struct BucketKey {
    int n, levels, align, bucket;
    bool operator<(const BucketKey &o) const
    {
        return n != o.n ? n < o.n : levels != o.levels ? levels < o.levels : align != o.align ? align < o.align
                                                                                             : bucket < o.bucket;
    }
};
std::mutex g_tune_mutex;
std::map<TuneKey, LaunchTune> g_tune_table;
std::map<BucketKey, LaunchTune> g_bucket_table;

BucketKey bucket_of(const TuneKey &k)
{
    return BucketKey{k.n, k.levels, k.align, (int)std::lround(2.0 * std::log2((double)k.w * k.h))};
}

// The shape for key k: its own, else its bucket's; false if neither exists.
bool tune_lookup(const TuneKey &k, LaunchTune *t)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it = g_tune_table.find(k);
    if (it != g_tune_table.end()) {
        *t = it->second;
        return true;
    }
    const auto bt = g_bucket_table.find(bucket_of(k));
    if (bt == g_bucket_table.end())
        return false;
    *t = bt->second;
    return true;
}

void tune_store(const TuneKey &k, const LaunchTune &t)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_table[k] = t;
    g_bucket_table[bucket_of(k)] = t;
}

TuneKey tune_key(int n, int w, int h, int levels, int64_t stride)
{
    return TuneKey{n, w, h, levels, stride % 16 == 0 ? 16 : (stride % 4 == 0 ? 4 : 1)};
}

bool shape_valid(const mtb_launch_shape &s)
{
    if (s.pyramid_slots_pct < 25 || s.pyramid_slots_pct > 400 || s.bitmaps_blocks_pct < 25 ||
        s.bitmaps_blocks_pct > 100)
        return false;
    if (s.pyramid_tile_group != 1 && s.pyramid_tile_group != 2 && s.pyramid_tile_group != 4)
        return false;
    if (s.bitmaps_waves != 2 && s.bitmaps_waves != 4 && s.bitmaps_waves != 8)
        return false;
    if (s.coarse_levels < -1 || s.coarse_levels > kCoarseLevels)
        return false;
    if (s.small_search < -1 || s.small_search > 1)
        return false;
    if (s.level1_from_level0 < -1 || s.level1_from_level0 > 1)
        return false;
    for (int l = 0; l < kMaxLevels; ++l) {
        const int r = s.search_rows[l], w = s.search_lanes[l];
        if (r != 0 && (r < kRowsStep || r > kRowsMax || r % kRowsStep != 0))
            return false;
        if (w != 0 && w != 8 && w != 16 && w != 32 && w != 64)
            return false;
    }
    return true;
}

LaunchTune from_shape(const mtb_launch_shape &s)
{
    LaunchTune t;
    t.pyr_pct = s.pyramid_slots_pct;
    t.pyr_group_log2 = s.pyramid_tile_group == 4 ? 2 : (s.pyramid_tile_group == 2 ? 1 : 0);
    t.bm_pct = s.bitmaps_blocks_pct;
    t.bm_waves = s.bitmaps_waves;
    t.coarse = s.coarse_levels;
    t.small = s.small_search;
    t.l1 = s.level1_from_level0;
    for (int l = 0; l < kMaxLevels; ++l) {
        t.rows[l] = s.search_rows[l];
        const int w = s.search_lanes[l];
        t.cw[l] = w == 8 ? 3 : w == 16 ? 4 : w == 32 ? 5 : w == 64 ? 6 : 0;
    }
    return t;
}

void to_shape(const LaunchTune &t, mtb_launch_shape *s)
{
    memset(s, 0, sizeof(*s));
    s->pyramid_slots_pct = t.pyr_pct;
    s->pyramid_tile_group = 1 << t.pyr_group_log2;
    s->bitmaps_blocks_pct = t.bm_pct;
    s->bitmaps_waves = t.bm_waves;
    s->coarse_levels = t.coarse;
    s->small_search = t.small;
    s->level1_from_level0 = t.l1;
    for (int l = 0; l < kMaxLevels; ++l) {
        s->search_rows[l] = t.rows[l];
        s->search_lanes[l] = t.cw[l] ? 1 << t.cw[l] : 0;
    }
}

// Device architecture and HIP runtime version that tuned shapes are valid for.
std::string tune_platform()
{
    int dev = 0, ver = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipRuntimeGetVersion(&ver) != hipSuccess)
        return std::string();
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos)
        arch.resize(colon);
    return arch + " hip-" + std::to_string(ver);
}

// Times candidate shapes for one key by the median of kReps calls of run(t)
// (HIP events on s, after a warm-up call), changing one knob at a time from
// the built-in shape and keeping a change only if it is at least 2 % faster.
// run(t) enqueues a whole call that uses shape t for this key.
template <typename Run>
mtb_status tune_one(const Geometry &g, int npairs, int cus, hipStream_t s, Run run, LaunchTune *out_best,
                    float *out_ms, float *out_default_ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return MTB_ERR_DEVICE;
    }
    constexpr int kReps = 7;
    auto time = [&](const LaunchTune &t, float *ms) -> mtb_status {
        mtb_status r = run(t);
        float v[kReps];
        for (int k = 0; k < kReps && r == MTB_OK; ++k) {
            if (hipEventRecord(e0, s) != hipSuccess)
                return MTB_ERR_DEVICE;
            r = run(t);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&v[k], e0, e1) != hipSuccess)
                return MTB_ERR_DEVICE;
        }
        if (r != MTB_OK)
            return r;
        std::sort(v, v + kReps);
        *ms = v[kReps / 2];
        return MTB_OK;
    };
    LaunchTune best;
    float best_ms = 0.f;
    mtb_status st = time(best, &best_ms);
    const float default_ms = best_ms;
    auto consider = [&](const LaunchTune &cand) {
        float ms = 0.f;
        if (st == MTB_OK)
            st = time(cand, &ms);
        if (st == MTB_OK && ms < 0.98f * best_ms) {
            best = cand;
            best_ms = ms;
        }
    };
    for (int pct : {50, 75, 150, 200}) {
        LaunchTune c = best;
        c.pyr_pct = pct;
        consider(c);
    }
    for (int gl : {1, 2}) {
        LaunchTune c = best;
        c.pyr_group_log2 = gl;
        consider(c);
    }
    for (int pct : {50, 75}) {
        LaunchTune c = best;
        c.bm_pct = pct;
        consider(c);
    }
    for (int w : {2, 8}) {
        LaunchTune c = best;
        c.bm_waves = w;
        consider(c);
    }
    if (npairs > 0 && small_search_fits(g)) {
        LaunchTune c = best;
        c.small = 0;
        consider(c);
    }
    for (int l1 : {0, 1}) {
        if (g.L < 2)
            break;
        LaunchTune c = best;
        c.l1 = l1;
        consider(c);
    }
    if (npairs > 0 && !small_search_used(g, &best)) {
        const int rule = coarse_level_count(g, npairs);
        const int most = g.L < kCoarseLevels ? g.L : kCoarseLevels;
        for (int cn : {rule - 1, rule + 1}) {
            if (cn < 0 || cn > most)
                continue;
            LaunchTune c = best;
            c.coarse = cn;
            consider(c);
        }
        for (int l = g.L - 1 - coarse_levels_used(g, npairs, &best); l >= 0; --l) {
            for (int cw : {3, 4, 5, 6}) {
                LaunchTune c = best;
                c.cw[l] = cw;
                consider(c);
            }
            const int r0 = search_rows_rule(g, l, npairs, cus, best.cw[l]);
            for (int r : {r0 / 2, 2 * r0}) {
                if (r < kRowsStep || r > kRowsMax || r % kRowsStep != 0)
                    continue;
                LaunchTune c = best;
                c.rows[l] = r;
                consider(c);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MTB_OK)
        return st;
    *out_best = best;
    *out_ms = best_ms;
    *out_default_ms = default_ms;
    return MTB_OK;
}

// One unit of a batch: the images of a pair item or a stack item (one size
// and row stride), its reference and its output rows.  A pair item (images
// reference, moving) writes one row, row0; a stack item writes row row0 + i
// for image i, zeros for its reference.
struct BatchUnit {
    const uint8_t *img[kMaxStack];
    int n = 0, ref = 0;
    int32_t W = 0, H = 0, L = 0;
    int64_t stride = 0;
    int row0 = 0;
    bool is_pair = false;
};

bool batch_item_valid(const mtb_batch_item &it, Geometry *g)
{
    return it.d_ref_rgb && it.d_mov_rgb && it.reserved == 0 && make_geometry(it.width, it.height, it.levels, g) &&
           it.row_stride >= 3 * (int64_t)it.width;
}

bool batch_stack_valid(const mtb_batch_stack &st, Geometry *g)
{
    if (!st.d_rgb || st.n < 1 || st.n > kMaxStack || st.ref_index < -1 || st.ref_index >= st.n || st.reserved != 0 ||
        st.row_stride < 3 * (int64_t)st.width || !make_geometry(st.width, st.height, st.levels, g))
        return false;
    for (int i = 0; i < st.n; ++i)
        if (!st.d_rgb[i])
            return false;
    return true;
}

// Units of valid pair items (item k writes row k), or of valid stack items
// (rows in item order, image by image); false if any item is invalid.
bool pair_units(const mtb_batch_item *it, int n, std::vector<BatchUnit> *u)
{
    u->assign(n, BatchUnit());
    Geometry g;
    for (int i = 0; i < n; ++i) {
        if (!batch_item_valid(it[i], &g))
            return false;
        BatchUnit &b = (*u)[i];
        b.img[0] = it[i].d_ref_rgb;
        b.img[1] = it[i].d_mov_rgb;
        b.n = 2;
        b.ref = 0;
        b.W = it[i].width;
        b.H = it[i].height;
        b.L = it[i].levels;
        b.stride = it[i].row_stride;
        b.row0 = i;
        b.is_pair = true;
    }
    return true;
}

bool stack_units(const mtb_batch_stack *st, int n, std::vector<BatchUnit> *u, int64_t *rows)
{
    u->assign(n, BatchUnit());
    Geometry g;
    int64_t row = 0;
    for (int i = 0; i < n; ++i) {
        if (!batch_stack_valid(st[i], &g))
            return false;
        BatchUnit &b = (*u)[i];
        for (int k = 0; k < st[i].n; ++k)
            b.img[k] = st[i].d_rgb[k];
        b.n = st[i].n;
        b.ref = st[i].ref_index < 0 ? st[i].n / 2 : st[i].ref_index;
        b.W = st[i].width;
        b.H = st[i].height;
        b.L = st[i].levels;
        b.stride = st[i].row_stride;
        b.row0 = (int)row;
        b.is_pair = false;
        row += st[i].n;
    }
    *rows = row;
    return true;
}

// Units of a batch that share one launch set: same geometry and stride, at
// most kMaxStack images together (16 pairs).
struct BatchGroup {
    int first;  // a unit of the group, for its geometry and stride
    std::vector<int> items;
    int images = 0;
};

// Splits a unit list into launch sets, in order of first appearance; a unit
// joins the open group of its size while the group's images stay within
// kMaxStack, else it opens a new one.
std::vector<BatchGroup> batch_groups(const std::vector<BatchUnit> &u)
{
    std::vector<BatchGroup> groups;
    std::vector<int> open;  // index into groups of the last group of each size seen
    for (int i = 0; i < (int)u.size(); ++i) {
        int found = -1;
        for (int k : open) {
            const BatchUnit &f = u[groups[k].first];
            if (f.W == u[i].W && f.H == u[i].H && f.L == u[i].L && f.stride == u[i].stride) {
                found = k;
                break;
            }
        }
        if (found >= 0 && groups[found].images + u[i].n > kMaxStack) {
            for (int &k : open)
                if (k == found)
                    k = (int)groups.size();
            groups.push_back(BatchGroup{i, {i}, u[i].n});
        } else if (found >= 0) {
            groups[found].items.push_back(i);
            groups[found].images += u[i].n;
        } else {
            open.push_back((int)groups.size());
            groups.push_back(BatchGroup{i, {i}, u[i].n});
        }
    }
    return groups;
}

// Pairs a group searches: every image of each unit but its reference.
int group_pairs(const std::vector<BatchUnit> &u, const BatchGroup &grp)
{
    int np = 0;
    for (int i : grp.items)
        np += u[i].n - 1;
    return np;
}

// The four quadrant pairs of a reference / moving pair as batch items
// (q = 0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right).
void quadrant_items(const uint8_t *ref, const uint8_t *mov, int32_t W, int32_t H, int64_t stride,
                    int32_t levels, mtb_batch_item *it)
{
    const int32_t w0 = W / 2, h0 = H / 2;
    for (int q = 0; q < 4; ++q) {
        const int32_t x = (q & 1) ? w0 : 0, y = (q & 2) ? h0 : 0;
        const int64_t off = (int64_t)y * stride + 3 * (int64_t)x;
        it[q].d_ref_rgb = ref ? ref + off : nullptr;
        it[q].d_mov_rgb = mov ? mov + off : nullptr;
        it[q].row_stride = stride;
        it[q].width = (q & 1) ? W - w0 : w0;
        it[q].height = (q & 2) ? H - h0 : h0;
        it[q].levels = levels;
        it[q].reserved = 0;
    }
}

// One pair's search (counters, bases, coarse surfaces, tickets) in the device
// buffer `state`, which is cleared first.
mtb_status align_pair_in(const void *d_bm_ref, const void *d_bm_mov, const Geometry &g, uint32_t *state,
                         int32_t *d_shift, uint32_t *d_err, uint32_t *d_trace, int32_t *d_level_shifts, int cus,
                         hipStream_t s)
{
    const int levels = g.L;

    // The one-workgroup search keeps no state in memory; the others count
    // into zeroed counters.
    if (!small_search_used(g, nullptr)) {
        ZeroArgs z;
        memset(&z, 0, sizeof(z));
        z.ptr[0] = state;
        z.words[0] = state_stride_words(levels) + kTicketWords;  // counters, bases, surfaces, tickets
        z.count = 1;
        if (launch_zero(z, s) != hipSuccess)
            return MTB_ERR_DEVICE;
    }

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

// ---- the allocation-free pair search (mtb_align_pair_scratch)

// One pair's search state and tickets for the most levels a call takes.
constexpr int64_t kPairScratchWords =
    (((int64_t)kMaxLevels * kCounterWords + 2 * kMaxLevels + kSurfWords + kAlign / 4 - 1) / (kAlign / 4)) *
        (kAlign / 4) +
    kTicketWords;

// A batch's groups run on up to kBatchLanes streams of the library at once
// (forked from and joined back to the caller's stream with events), each
// lane with its own workspace range: while one group's search, a chain of
// short latency-bound launches, leaves the device mostly idle, another
// group's bandwidth-bound passes fill it.
constexpr int kBatchLanes = 4;

struct BatchPlan {
    std::vector<BatchGroup> groups;
    std::vector<int> lane;   // lane of each group
    int lanes = 1;
    int64_t lane_bytes = 0;  // workspace bytes of one lane (256-byte multiple)
};

BatchPlan batch_plan(const std::vector<BatchUnit> &u)
{
    BatchPlan p;
    p.groups = batch_groups(u);
    const int ng = (int)p.groups.size();
    p.lanes = ng < kBatchLanes ? ng : kBatchLanes;
    std::vector<int64_t> px(ng);
    for (int k = 0; k < ng; ++k) {
        const BatchUnit &f = u[p.groups[k].first];
        Geometry g;
        make_geometry(f.W, f.H, f.L, &g);
        const int64_t b = align_up(set_workspace_bytes(g, p.groups[k].images, group_pairs(u, p.groups[k])), kAlign);
        p.lane_bytes = b > p.lane_bytes ? b : p.lane_bytes;
        px[k] = (int64_t)f.W * f.H * p.groups[k].images;
    }
    // Largest groups first, each to the lane with the fewest pixels so far.
    std::vector<int> order(ng);
    for (int k = 0; k < ng; ++k)
        order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return px[a] > px[b]; });
    std::vector<int64_t> load(p.lanes, 0);
    p.lane.assign(ng, 0);
    for (int k : order) {
        int best = 0;
        for (int l = 1; l < p.lanes; ++l)
            if (load[l] < load[best])
                best = l;
        p.lane[k] = best;
        load[best] += px[k];
    }
    return p;
}

// The library's lane streams and events of the calling thread on the current
// device (created once, at default priority, kept until the process ends).
struct Lanes {
    int device = -1;
    hipStream_t s[kBatchLanes] = {};
    hipEvent_t fork = nullptr, done[kBatchLanes] = {};
};
thread_local std::vector<Lanes> t_lanes;

Lanes *batch_lanes()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return nullptr;
    for (Lanes &l : t_lanes)
        if (l.device == dev)
            return &l;
    Lanes l;
    l.device = dev;
    bool ok = hipEventCreateWithFlags(&l.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kBatchLanes && ok; ++i)
        ok = hipStreamCreateWithFlags(&l.s[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&l.done[i], hipEventDisableTiming) == hipSuccess;
    if (!ok)
        return nullptr;
    t_lanes.push_back(l);
    return &t_lanes.back();
}

// A batch: one launch set per group of units that share geometry and stride,
// each with its key's tuned shape (or, for the key ov_key, the shape ov_shape);
// rows output rows.  Units must be valid.
mtb_status align_units(const std::vector<BatchUnit> &u, int64_t rows, int32_t exclude_range, void *d_workspace,
                       size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs, hipStream_t s,
                       const TuneKey *ov_key, const LaunchTune *ov_shape)
{
    if (!d_workspace || !d_shifts || !d_errs || exclude_range < 0 || exclude_range > 255)
        return MTB_ERR_INVALID_ARG;
    const BatchPlan plan = batch_plan(u);
    if (workspace_bytes < (size_t)(plan.lanes * plan.lane_bytes + kAlign))
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    uint8_t *ws = (uint8_t *)align_up((int64_t)(uintptr_t)d_workspace, kAlign);
    // A stack item's reference rows are written by no search: clear every
    // row first, on the caller's stream, before the lanes fork from it.
    bool stacks = false;
    for (const BatchUnit &b : u)
        stacks = stacks || !b.is_pair;
    if (stacks) {
        ZeroArgs z;
        memset(&z, 0, sizeof(z));
        z.ptr[0] = (uint32_t *)d_shifts;
        z.words[0] = 2 * rows;
        z.ptr[1] = d_errs;
        z.words[1] = rows;
        z.count = 2;
        if (launch_zero(z, s) != hipSuccess)
            return MTB_ERR_DEVICE;
    }
    Lanes *lanes = plan.lanes > 1 ? batch_lanes() : nullptr;
    if (plan.lanes > 1 && !lanes)
        return MTB_ERR_DEVICE;
    if (lanes) {
        if (hipEventRecord(lanes->fork, s) != hipSuccess)
            return MTB_ERR_DEVICE;
        for (int l = 0; l < plan.lanes; ++l)
            if (hipStreamWaitEvent(lanes->s[l], lanes->fork, 0) != hipSuccess)
                return MTB_ERR_DEVICE;
    }
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < plan.groups.size() && e == hipSuccess; ++k) {
        const BatchGroup &grp = plan.groups[k];
        if (group_pairs(u, grp) == 0)
            continue;  // single-image stacks only: their rows are the zeros above
        const BatchUnit &f = u[grp.first];
        Geometry g;
        make_geometry(f.W, f.H, f.L, &g);
        PairSet ps;
        int align = 16;
        for (int item : grp.items) {
            const BatchUnit &b = u[item];
            const int base = ps.n;
            for (int i = 0; i < b.n; ++i) {
                ps.rgb[ps.n++] = b.img[i];
                const int a = row_alignment(b.img[i], b.stride);
                align = a < align ? a : align;
            }
            for (int i = 0; i < b.n; ++i) {
                if (i == b.ref)
                    continue;
                ps.ref_img[ps.npairs] = base + b.ref;
                ps.mov_img[ps.npairs] = base + i;
                ps.out_row[ps.npairs++] = b.is_pair ? b.row0 : b.row0 + i;
            }
        }
        SearchOutputs out;
        memset(&out, 0, sizeof(out));
        out.n_out = (int32_t)rows;
        out.shifts = d_shifts;
        out.errs = d_errs;
        ZeroArgs z;
        memset(&z, 0, sizeof(z));
        const TuneKey key = tune_key(ps.n, f.W, f.H, f.L, f.stride);
        LaunchTune t;
        if (ov_key && *ov_key == key)
            t = *ov_shape;
        else
            tune_lookup(key, &t);
        const int l = plan.lane[k];
        e = enqueue_set(ps, g, f.stride, align, exclude_range, ws + l * plan.lane_bytes, out, z, cus,
                        lanes ? lanes->s[l] : s, false, t);
    }
    // Join every lane back into the caller's stream, also after a failed
    // launch, so that later work on it follows everything enqueued here.
    bool joined = true;
    if (lanes)
        for (int l = 0; l < plan.lanes; ++l)
            joined = hipEventRecord(lanes->done[l], lanes->s[l]) == hipSuccess &&
                     hipStreamWaitEvent(s, lanes->done[l], 0) == hipSuccess && joined;
    return e == hipSuccess && joined ? MTB_OK : MTB_ERR_DEVICE;
}

// The pair-item batch.
mtb_status align_batch(const mtb_batch_item *h_items, int32_t n_items, int32_t exclude_range, void *d_workspace,
                       size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs, hipStream_t s,
                       const TuneKey *ov_key, const LaunchTune *ov_shape)
{
    std::vector<BatchUnit> u;
    if (!h_items || n_items < 1 || n_items > MTB_MAX_BATCH || !pair_units(h_items, n_items, &u))
        return MTB_ERR_INVALID_ARG;
    return align_units(u, n_items, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs, s, ov_key,
                       ov_shape);
}

}  // namespace

// The search state of mtb_align_pair_scratch: one copy per device, held until
// the process ends, shared by every call on that device (calls that overlap
// on one device race on it).  Host code never passes this name to a kernel:
// it is a host-side stand-in; device_scratch() gives the device address.
static __device__ __align__(256) uint32_t scratch[kPairScratchWords];

namespace {

std::mutex g_scratch_mutex;
uint32_t *g_scratch_ptr[64];

// Device address of `scratch` on the current device, looked up once per
// device with that device current; null if the lookup fails.
uint32_t *device_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return nullptr;
        g_scratch_ptr[dev] = (uint32_t *)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

void note_pyramid_launch(int blocks, int merged)
{
    t_pyr_blocks = blocks;
    t_pyr_merged = merged;
}

bool injected_launch_failure()
{
    if (t_fail_after < 0)
        return false;
    if (t_fail_after-- == 0)
        return true;  // t_fail_after is now -1: one failure only
    return false;
}

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
    return (size_t)(set_workspace_bytes(g, n, n - 1) + kAlign);
}

mtb_status mtb_stack_image_buffers(const void *d_workspace, int32_t n, int32_t width, int32_t height,
                                   int32_t levels, void **h_pyramids, void **h_bitmaps)
{
    Geometry g;
    if (!d_workspace || !h_pyramids || !h_bitmaps || n < 1 || n > kMaxStack ||
        !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    uint8_t *ws = (uint8_t *)align_up((int64_t)(uintptr_t)d_workspace, kAlign);
    for (int i = 0; i < n; ++i) {
        h_pyramids[i] = ws + i * g.pyramid_bytes;
        h_bitmaps[i] = ws + n * g.pyramid_bytes + i * g.bitmaps_bytes;
    }
    return MTB_OK;
}

int32_t mtb_level1_from_level0(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels)
{
    Geometry g;
    if (n < 1 || n > kMaxStack || row_stride < 3 * (int64_t)width || !make_geometry(width, height, levels, &g))
        return -1;
    LaunchTune t;
    tune_lookup(tune_key(n, width, height, levels, row_stride), &t);
    return level1_from_level0(g, n, t) ? 1 : 0;
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
    z.words[0] = (g.pyramid_bytes - g.hist_off) / 4;  // histograms and merge scratch
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
    return align_pair_in(d_bm_ref, d_bm_mov, g, (uint32_t *)d_workspace, d_shift, d_err, d_trace, d_level_shifts,
                         cus, (hipStream_t)stream);
}

mtb_status mtb_align_pair_scratch(const void *d_bm_ref, const void *d_bm_mov, int32_t width,
                                  int32_t height, int32_t levels, int32_t *d_shift, uint32_t *d_err,
                                  uint32_t *d_trace, int32_t *d_level_shifts, void *stream)
{
    Geometry g;
    if (!d_bm_ref || !d_bm_mov || !d_shift || !d_err || !make_geometry(width, height, levels, &g))
        return MTB_ERR_INVALID_ARG;
    // The array holds the state of MTB_MAX_LEVELS levels, the most any call takes.
    if (state_stride_words(levels) + kTicketWords > kPairScratchWords)
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    uint32_t *state = device_scratch();
    if (!state)
        return MTB_ERR_DEVICE;
    return align_pair_in(d_bm_ref, d_bm_mov, g, state, d_shift, d_err, d_trace, d_level_shifts, cus,
                         (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Both stack modes: every image against the reference, or (chained) every
// image against its neighbour towards the reference, the shifts then summed.
mtb_status align_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width, int32_t height,
                       int64_t row_stride, int32_t levels, int32_t exclude_range, int32_t ref_index,
                       void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                       uint32_t *d_trace, bool chained, hipStream_t s, bool bytemaps = false,
                       const LaunchTune *shape = nullptr)
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
    const size_t need = bytemaps ? mtb_stack_bytemaps_workspace_bytes(n, width, height, levels)
                                 : mtb_stack_workspace_bytes(n, width, height, levels);
    if (workspace_bytes < need)
        return MTB_ERR_WORKSPACE;
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;

    PairSet ps;
    for (int i = 0; i < n; ++i) {
        ps.rgb[i] = h_d_rgb[i];
        if (i != ref) {
            ps.ref_img[ps.npairs] = chained ? (i < ref ? i + 1 : i - 1) : ref;
            ps.mov_img[ps.npairs] = i;
            ps.out_row[ps.npairs++] = i;
        }
    }
    ps.n = n;
    SearchOutputs out;
    memset(&out, 0, sizeof(out));
    out.n_out = n;
    out.shifts = d_shifts;
    out.errs = d_errs;
    out.trace = d_trace;
    // The reference's output rows stay zero; the search writes every other row.
    ZeroArgs z;
    memset(&z, 0, sizeof(z));
    z.ptr[z.count] = (uint32_t *)d_shifts;
    z.words[z.count++] = 2 * (int64_t)n;
    z.ptr[z.count] = d_errs;
    z.words[z.count++] = n;
    if (d_trace) {
        z.ptr[z.count] = d_trace;
        z.words[z.count++] = 9 * (int64_t)levels * n;
    }
    uint8_t *ws = (uint8_t *)align_up((int64_t)(uintptr_t)d_workspace, kAlign);
    LaunchTune t;
    if (shape)
        t = *shape;
    else if (!bytemaps)
        tune_lookup(tune_key(n, width, height, levels, row_stride), &t);
    hipError_t e = enqueue_set(ps, g, row_stride, align, exclude_range, ws, out, z, cus, s, bytemaps, t);
    if (e == hipSuccess && chained && n > 1)
        e = launch_chain(d_shifts, n, ref, s);
    return device_status(e);
}

}  // namespace

extern "C" {

mtb_status mtb_align_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                           int32_t height, int64_t row_stride, int32_t levels,
                           int32_t exclude_range, int32_t ref_index, void *d_workspace,
                           size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                           uint32_t *d_trace, void *stream)
{
    return align_stack(h_d_rgb, n, width, height, row_stride, levels, exclude_range, ref_index, d_workspace,
                       workspace_bytes, d_shifts, d_errs, d_trace, false, (hipStream_t)stream);
}

size_t mtb_stack_bytemaps_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t levels)
{
    Geometry g;
    if (n < 1 || n > kMaxStack || !make_geometry(width, height, levels, &g))
        return 0;
    return (size_t)(set_workspace_bytes(g, n, n - 1, true) + kAlign);
}

mtb_status mtb_align_stack_bytemaps(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                                    int32_t height, int64_t row_stride, int32_t levels,
                                    int32_t exclude_range, int32_t ref_index, void *d_workspace,
                                    size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                                    uint32_t *d_trace, void *stream)
{
    return align_stack(h_d_rgb, n, width, height, row_stride, levels, exclude_range, ref_index, d_workspace,
                       workspace_bytes, d_shifts, d_errs, d_trace, false, (hipStream_t)stream, true);
}

mtb_status mtb_align_stack_chained(const uint8_t *const *h_d_rgb, int32_t n, int32_t width,
                                   int32_t height, int64_t row_stride, int32_t levels,
                                   int32_t exclude_range, int32_t ref_index, void *d_workspace,
                                   size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                                   uint32_t *d_trace, void *stream)
{
    return align_stack(h_d_rgb, n, width, height, row_stride, levels, exclude_range, ref_index, d_workspace,
                       workspace_bytes, d_shifts, d_errs, d_trace, true, (hipStream_t)stream);
}

mtb_status mtb_tune_stack(const uint8_t *const *h_d_rgb, int32_t n, int32_t width, int32_t height,
                          int64_t row_stride, int32_t levels, int32_t exclude_range, int32_t ref_index,
                          void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                          void *stream, mtb_launch_shape *h_out)
{
    if (!h_out)
        return MTB_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    auto run = [&](const LaunchTune &t) {
        return align_stack(h_d_rgb, n, width, height, row_stride, levels, exclude_range, ref_index, d_workspace,
                           workspace_bytes, d_shifts, d_errs, nullptr, false, s, false, &t);
    };
    mtb_status st = run(LaunchTune());  // validates every argument before anything is timed
    if (st != MTB_OK)
        return st;
    Geometry g;
    make_geometry(width, height, levels, &g);  // valid: the first run checked it
    LaunchTune best;
    float best_ms = 0.f, default_ms = 0.f;
    st = tune_one(g, n - 1, current_device_cus(), s, run, &best, &best_ms, &default_ms);
    if (st != MTB_OK)
        return st;
    // The winning shape leaves its results in d_shifts / d_errs as well.
    st = run(best);
    if (st != MTB_OK)
        return st;
    tune_store(tune_key(n, width, height, levels, row_stride), best);
    to_shape(best, h_out);
    h_out->step_ms = best_ms;
    h_out->default_ms = default_ms;
    return MTB_OK;
}

mtb_status mtb_set_shape(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels,
                         const mtb_launch_shape *shape)
{
    Geometry g;
    if (!shape || n < 1 || n > kMaxStack || row_stride < 3 * (int64_t)width || !make_geometry(width, height, levels, &g) ||
        !shape_valid(*shape))
        return MTB_ERR_INVALID_ARG;
    tune_store(tune_key(n, width, height, levels, row_stride), from_shape(*shape));
    return MTB_OK;
}

mtb_status mtb_tuned_shape(int32_t n, int32_t width, int32_t height, int64_t row_stride, int32_t levels,
                           mtb_launch_shape *h_out)
{
    LaunchTune t;
    if (!h_out || !tune_lookup(tune_key(n, width, height, levels, row_stride), &t))
        return MTB_ERR_INVALID_ARG;
    to_shape(t, h_out);
    return MTB_OK;
}

mtb_status mtb_test_last_pyramid(int32_t *h_blocks, int32_t *h_merged)
{
    if (!h_blocks || !h_merged || t_pyr_blocks < 0)
        return MTB_ERR_INVALID_ARG;
    *h_blocks = t_pyr_blocks;
    *h_merged = t_pyr_merged;
    return MTB_OK;
}

mtb_status mtb_test_fail_launch(int32_t after)
{
    t_fail_after = after < 0 ? -1 : after;
    return MTB_OK;
}

void mtb_tune_reset(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_table.clear();
    g_bucket_table.clear();
}

mtb_status mtb_tune_save(const char *path)
{
    if (!path)
        return MTB_ERR_INVALID_ARG;
    const std::string platform = tune_platform();
    if (platform.empty())
        return MTB_ERR_UNSUPPORTED;
    FILE *f = fopen(path, "w");
    if (!f)
        return MTB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    bool ok = fprintf(f, "mtb-tune 3 %s\n", platform.c_str()) > 0;
    for (const auto &kv : g_tune_table) {
        const TuneKey &k = kv.first;
        const LaunchTune &t = kv.second;
        ok = ok && fprintf(f, "%d %d %d %d %d  %d %d %d %d %d %d %d ", k.n, k.w, k.h, k.levels, k.align, t.pyr_pct,
                           t.pyr_group_log2, t.bm_pct, t.bm_waves, t.coarse, t.small, t.l1) > 0;
        for (int l = 0; l < kMaxLevels && ok; ++l)
            ok = fprintf(f, " %d", t.rows[l]) > 0;
        for (int l = 0; l < kMaxLevels && ok; ++l)
            ok = fprintf(f, " %d", t.cw[l]) > 0;
        ok = ok && fprintf(f, "\n") > 0;
    }
    ok = (fclose(f) == 0) && ok;
    return ok ? MTB_OK : MTB_ERR_INVALID_ARG;
}

mtb_status mtb_tune_load(const char *path, int32_t *h_loaded)
{
    if (!path || !h_loaded)
        return MTB_ERR_INVALID_ARG;
    *h_loaded = 0;
    const std::string platform = tune_platform();
    if (platform.empty())
        return MTB_ERR_UNSUPPORTED;
    FILE *f = fopen(path, "r");
    if (!f)
        return MTB_ERR_INVALID_ARG;
    char line[1024];
    std::vector<std::pair<TuneKey, LaunchTune>> got;
    bool ok = fgets(line, sizeof(line), f) != nullptr;
    // Shapes tuned on another architecture or HIP runtime are skipped whole.
    const bool same = ok && std::string(line) == "mtb-tune 3 " + platform + "\n";
    while (ok && same && fgets(line, sizeof(line), f)) {
        TuneKey k;
        LaunchTune t;
        int used = 0;
        const char *p = line;
        ok = sscanf(p, "%d %d %d %d %d %d %d %d %d %d %d %d%n", &k.n, &k.w, &k.h, &k.levels, &k.align, &t.pyr_pct,
                    &t.pyr_group_log2, &t.bm_pct, &t.bm_waves, &t.coarse, &t.small, &t.l1, &used) == 12;
        p += used;
        for (int l = 0; l < 2 * kMaxLevels && ok; ++l) {
            ok = sscanf(p, "%d%n", l < kMaxLevels ? &t.rows[l] : &t.cw[l - kMaxLevels], &used) == 1;
            p += used;
        }
        if (!ok)
            break;
        mtb_launch_shape sh;
        to_shape(t, &sh);
        Geometry g;
        ok = k.n >= 1 && k.n <= kMaxStack && (k.align == 1 || k.align == 4 || k.align == 16) &&
             t.pyr_group_log2 >= 0 && t.pyr_group_log2 <= 2 && shape_valid(sh) &&
             make_geometry(k.w, k.h, k.levels, &g);
        for (int l = 0; l < kMaxLevels && ok; ++l)
            ok = t.cw[l] == 0 || (t.cw[l] >= 3 && t.cw[l] <= 6);
        if (ok)
            got.push_back({k, t});
    }
    fclose(f);
    if (!ok)
        return MTB_ERR_INVALID_ARG;
    for (const auto &kv : got)
        tune_store(kv.first, kv.second);
    *h_loaded = (int32_t)got.size();
    return MTB_OK;
}

mtb_status mtb_apply_shifts(const uint8_t *const *h_d_rgb, int32_t n, int32_t width, int32_t height,
                            int64_t row_stride, const int32_t *d_shifts, int32_t fill,
                            uint8_t *const *h_d_out, int64_t out_stride, void *stream)
{
    if (!h_d_rgb || !h_d_out || !d_shifts || n < 1 || n > kMaxStack || width < 1 || height < 1 ||
        (int64_t)width * height >= ((int64_t)1 << 31))
        return MTB_ERR_INVALID_ARG;
    if (row_stride < 3 * (int64_t)width || out_stride < 3 * (int64_t)width || (fill != 0 && fill != 1))
        return MTB_ERR_INVALID_ARG;
    ApplyArgs a;
    memset(&a, 0, sizeof(a));
    bool aligned = row_stride % 4 == 0 && out_stride % 16 == 0;
    for (int i = 0; i < n; ++i) {
        if (!h_d_rgb[i] || !h_d_out[i])
            return MTB_ERR_INVALID_ARG;
        a.rgb[i] = h_d_rgb[i];
        a.out[i] = h_d_out[i];
        aligned = aligned && (uintptr_t)h_d_rgb[i] % 4 == 0 && (uintptr_t)h_d_out[i] % 16 == 0;
    }
    const int cus = current_device_cus();
    if (cus <= 0)
        return MTB_ERR_UNSUPPORTED;
    a.shifts = d_shifts;
    a.stride = row_stride;
    a.out_stride = out_stride;
    a.n = n;
    a.width = width;
    a.height = height;
    a.fill = fill;
    a.aligned = aligned ? 1 : 0;
    return device_status(launch_apply(a, cus, (hipStream_t)stream));
}

mtb_status mtb_stage_rgb(const uint8_t *h_rgb, int64_t src_stride, int32_t width, int32_t height,
                         uint8_t *d_rgb, int64_t dst_stride, void *stream)
{
    if (!h_rgb || !d_rgb || width < 1 || height < 1 || (int64_t)width * height >= ((int64_t)1 << 31))
        return MTB_ERR_INVALID_ARG;
    if (src_stride < 3 * (int64_t)width || dst_stride < 3 * (int64_t)width)
        return MTB_ERR_INVALID_ARG;
    return device_status(hipMemcpy2DAsync(d_rgb, (size_t)dst_stride, h_rgb, (size_t)src_stride,
                                          3 * (size_t)width, (size_t)height, hipMemcpyHostToDevice,
                                          (hipStream_t)stream));
}

size_t mtb_batch_workspace_bytes(const mtb_batch_item *h_items, int32_t n_items)
{
    std::vector<BatchUnit> u;
    if (!h_items || n_items < 1 || n_items > MTB_MAX_BATCH || !pair_units(h_items, n_items, &u))
        return 0;
    const BatchPlan plan = batch_plan(u);
    return (size_t)(plan.lanes * plan.lane_bytes + kAlign);
}

size_t mtb_batch_stacks_workspace_bytes(const mtb_batch_stack *h_items, int32_t n_items)
{
    std::vector<BatchUnit> u;
    int64_t rows = 0;
    if (!h_items || n_items < 1 || n_items > MTB_MAX_BATCH || !stack_units(h_items, n_items, &u, &rows))
        return 0;
    const BatchPlan plan = batch_plan(u);
    return (size_t)(plan.lanes * plan.lane_bytes + kAlign);
}

mtb_status mtb_align_batch_stacks(const mtb_batch_stack *h_items, int32_t n_items, int32_t exclude_range,
                                  void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                                  void *stream)
{
    std::vector<BatchUnit> u;
    int64_t rows = 0;
    if (!h_items || n_items < 1 || n_items > MTB_MAX_BATCH || !stack_units(h_items, n_items, &u, &rows))
        return MTB_ERR_INVALID_ARG;
    return align_units(u, rows, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs, (hipStream_t)stream,
                       nullptr, nullptr);
}

mtb_status mtb_align_batch(const mtb_batch_item *h_items, int32_t n_items, int32_t exclude_range,
                           void *d_workspace, size_t workspace_bytes, int32_t *d_shifts,
                           uint32_t *d_errs, void *stream)
{
    return align_batch(h_items, n_items, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs,
                       (hipStream_t)stream, nullptr, nullptr);
}

mtb_status mtb_tune_batch(const mtb_batch_item *h_items, int32_t n_items, int32_t exclude_range,
                          void *d_workspace, size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                          void *stream, int32_t *h_tuned)
{
    if (!h_tuned)
        return MTB_ERR_INVALID_ARG;
    *h_tuned = 0;
    const hipStream_t s = (hipStream_t)stream;
    mtb_status st = align_batch(h_items, n_items, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs, s,
                                nullptr, nullptr);  // validates every argument first
    if (st != MTB_OK)
        return st;
    // One group key after another: the whole batch is timed with candidate
    // shapes for that key, the other keys at their current shapes.
    std::vector<TuneKey> done;
    std::vector<BatchUnit> u;
    pair_units(h_items, n_items, &u);  // valid: the call above checked every item
    for (const BatchGroup &grp : batch_groups(u)) {
        const BatchUnit &f = u[grp.first];
        const TuneKey key = tune_key(grp.images, f.W, f.H, f.L, f.stride);
        if (std::find(done.begin(), done.end(), key) != done.end())
            continue;
        done.push_back(key);
        Geometry g;
        make_geometry(f.W, f.H, f.L, &g);
        auto run = [&](const LaunchTune &t) {
            return align_batch(h_items, n_items, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs, s,
                               &key, &t);
        };
        LaunchTune best;
        float ms = 0.f, def = 0.f;
        st = tune_one(g, group_pairs(u, grp), current_device_cus(), s, run, &best, &ms, &def);
        if (st != MTB_OK)
            return st;
        tune_store(key, best);
        ++*h_tuned;
    }
    return align_batch(h_items, n_items, exclude_range, d_workspace, workspace_bytes, d_shifts, d_errs, s, nullptr,
                       nullptr);
}

size_t mtb_quadrant_workspace_bytes(int32_t width, int32_t height, int64_t row_stride, int32_t levels)
{
    if (width < 2 || height < 2 || row_stride < 3 * (int64_t)width)
        return 0;
    mtb_batch_item it[4];
    const uint8_t *fake = (const uint8_t *)(uintptr_t)kAlign;  // sizes only; never dereferenced
    quadrant_items(fake, fake, width, height, row_stride, levels, it);
    return mtb_batch_workspace_bytes(it, 4);
}

mtb_status mtb_align_quadrants(const uint8_t *d_ref_rgb, const uint8_t *d_mov_rgb, int32_t width,
                               int32_t height, int64_t row_stride, int32_t levels,
                               int32_t exclude_range, int32_t tolerance, void *d_workspace,
                               size_t workspace_bytes, int32_t *d_shifts, uint32_t *d_errs,
                               int32_t *d_flag, void *stream)
{
    if (!d_ref_rgb || !d_mov_rgb || !d_flag || tolerance < 0 || width < 2 || height < 2 ||
        row_stride < 3 * (int64_t)width)
        return MTB_ERR_INVALID_ARG;
    mtb_batch_item it[4];
    quadrant_items(d_ref_rgb, d_mov_rgb, width, height, row_stride, levels, it);
    const size_t need = mtb_batch_workspace_bytes(it, 4);
    if (need == 0)
        return MTB_ERR_INVALID_ARG;
    if (workspace_bytes < need)
        return MTB_ERR_WORKSPACE;
    const mtb_status st = mtb_align_batch(it, 4, exclude_range, d_workspace, workspace_bytes, d_shifts,
                                          d_errs, stream);
    if (st != MTB_OK)
        return st;
    return device_status(launch_quadrant_flag(d_shifts, tolerance, d_flag, (hipStream_t)stream));
}

}  // extern "C"
