// mtb_internal.h -- layout arithmetic and kernel argument blocks shared by the
// HIP kernels (mtb_kernels.hip) and the C-ABI entry points (mtb_api.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mtb.h"

namespace mtb {

constexpr int kMaxLevels = MTB_MAX_LEVELS;
constexpr int kMaxStack = MTB_MAX_STACK;
constexpr int kAlign = 256;

// Pass 1 fuses this many pyramid levels per workgroup tile; the tile is
// kTileH = 2^(kFused-1) rows by kTileW columns of level 0.
constexpr int kFused = 7;
// Accelerator complex dies (XCDs) of the device, each with its own L2.
constexpr int kXcds = 8;
// k_pyramid's histogram merge scratch per image: one uint32[kFused][256] copy
// per XCD, then kXcds tile tickets and one XCD ticket.  It follows the
// histograms, so that one range from hist_off to the end of the pyramid
// buffer clears both.
constexpr int64_t kHMergeWords = (int64_t)kXcds * kFused * 256 + 64;
// Launches with at least this many workgroups per image merge histograms
// through the per-XCD copies.
constexpr int kMergeMinWgsPerImage = 192;
constexpr int kTileH = 64;
constexpr int kTileW = 256;

// Search counters are spread over this many copies per (pair, level) so that
// concurrent workgroups do not all add into the same nine words.
constexpr int kCopies = 16;
// Per pair and level: kCopies x 9 uint32 counters.
constexpr int kCounterWords = kCopies * 9;

inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Geometry of one pyramid level, with offsets into the per-image buffers.
struct LevelGeom {
    int32_t w, h;         // level size in pixels
    int32_t wpr;          // uint64 words per bitmap row = 2 * ceil(w / 128)
    int32_t pad_;
    int64_t gray_off;     // bytes, pyramid buffer
    int64_t gray_pitch;   // bytes = 64 * wpr, a multiple of 128
    int64_t tb_off;       // bytes, bitmaps buffer
    int64_t eb_off;       // bytes, bitmaps buffer
    int64_t bt_off;       // bytes, byte-maps buffer: T as 255/0 bytes, rows of gray_pitch
    int64_t be_off;       // bytes, byte-maps buffer: E likewise
};

struct Geometry {
    int32_t W, H, L, pad_;
    LevelGeom lv[kMaxLevels];
    int64_t hist_off;       // uint32[L][256] in the pyramid buffer
    int64_t hmerge_off;     // pyramid buffer: k_pyramid's histogram merge scratch (kHMergeWords)
    int64_t pyramid_bytes;
    int64_t med_off;        // int32[L] in the bitmaps buffer
    int64_t bitmaps_bytes;
    int64_t bmed_off;       // int32[L] in the byte-maps buffer
    int64_t bytemaps_bytes;
};

// Returns false if the size or level count is out of range.
bool make_geometry(int32_t W, int32_t H, int32_t L, Geometry *g);
int32_t max_levels(int32_t W, int32_t H);

// ------------------------------------------------------------------ pass 1

struct PyramidArgs {
    const uint8_t *rgb[kMaxStack];
    uint8_t *pyr[kMaxStack];
    int64_t stride;          // bytes between RGB rows
    int32_t n;               // images
    int32_t tiles_x, tiles_y;
    int32_t xcd_tiles;       // tiles of each XCD's contiguous share of the work
    int32_t align;           // 16, 4 or 1: alignment every RGB row start is known to have
    int32_t merge;           // 1: histograms merged through per-XCD copies (see k_pyramid)
    int32_t group_log2;      // a workgroup takes 2^group_log2 consecutive tiles of a row at a time
    int32_t skip_l1;         // 1: level 1's gray is not stored (the bitmaps pass forms it from level 0)
    Geometry g;
};

// Levels kFused..L-1 are built from level kFused-1 by one workgroup per image.
struct CoarsePyramidArgs {
    uint8_t *pyr[kMaxStack];
    int32_t n, pad_;
    Geometry g;
};

// ------------------------------------------------------------------ pass 2

// The bitmaps pass walks each level as a flat run of 64-pixel words, in
// chunks of kChunkWords words (kChunkWords * 64 gray bytes) per wavefront.
constexpr int kChunkWords = 32;
// With `pairs` set, level 0 is walked instead in units of two rows by
// kPairWords words, and each unit also yields the level-1 bitmaps below it
// (level 1 then has no chunks of its own and its gray is not read).
constexpr int kPairWords = 16;

struct BitmapArgs {
    const uint8_t *pyr[kMaxStack];
    uint8_t *bm[kMaxStack];
    int32_t n;
    int32_t exclude;
    int32_t pairs;   // 1: levels 0 and 1 from level 0's gray, in two-row units
    int32_t pad_;
    int64_t chunk_start[kMaxLevels + 1];  // first chunk (or unit) of each level within one image
    Geometry g;
};

// ------------------------------------------------------------------ search

// The coarsest levels (at most kCoarseLevels) are searched exhaustively over
// every shift the coarse-to-fine search could reach there: radius 2^(i+1) - 1
// at the i-th coarsest level.  Their error surfaces take kSurfWords words; the
// first kLdsSurfWords (the windows of radius 1, 3 and 7) are staged in LDS by
// the walk, the larger ones read from memory.
constexpr int kCoarseLevels = 5;
constexpr int kSurfWords = 3 * 3 + 7 * 7 + 15 * 15 + 31 * 31 + 63 * 63;
constexpr int kLdsSurfWords = 3 * 3 + 7 * 7 + 15 * 15;

// Per pair the search state is: counters uint32[L][kCounterWords], then
// base int32[L][2] (the centre of each level's nine candidates), then the
// coarse error surfaces uint32[kSurfWords].  After every pair's state come the
// ticket counters of the coarse launch and of the level-0 launch: each
// kTicketGroups group counters and one counter of completed groups.
inline int64_t pair_state_words(int32_t L) { return (int64_t)L * kCounterWords + 2 * L + kSurfWords; }
constexpr int kTicketGroups = 32;
constexpr int kTicketWords = 2 * (kTicketGroups + 1);

// Where the search writes its results; the last workgroup of the launch
// that searches level 0 fills them in.
struct SearchOutputs {
    int32_t pair_image[kMaxStack];   // output row of each pair (stack index)
    int32_t n_out;                   // rows of the outputs
    int32_t pad_;
    int32_t *shifts;                 // [n_out][2]
    uint32_t *errs;                  // [n_out]
    uint32_t *trace;                 // NULL or [n_out][L][9]
    int32_t *level_shifts;           // NULL or [n_out][L][2]
};

struct SearchArgs {
    const uint8_t *ref[kMaxStack];   // bitmaps buffer of each pair's reference
    const uint8_t *mov[kMaxStack];   // bitmaps buffer of each pair's moving image
    uint32_t *state;                 // pair p's state at state + p * state_stride
    uint32_t *done;                  // ticket counters: coarse launch, then level-0 launch
    int64_t state_stride;            // uint32 words
    int32_t npairs;
    int32_t level;                   // fine kernel: the level searched
    int32_t coarse_n;                // levels L-1 .. L-coarse_n searched exhaustively
    int32_t rows_per_stream;         // rows per lane in one work unit
    int32_t cw_log2;                 // fine kernel: lanes per row stream (log2, 3..6), 0: the rule
    int32_t pad_;
    SearchOutputs out;
    Geometry g;
};

// ------------------------------------------------------------------ apply shifts

// Translating each image of a stack by its shift (out[y][x] = in[y - dy][x - dx]).
struct ApplyArgs {
    const uint8_t *rgb[kMaxStack];
    uint8_t *out[kMaxStack];
    const int32_t *shifts;  // device int32[n][2]
    int64_t stride, out_stride;
    int32_t n, width, height;
    int32_t fill;           // 0: zeros outside the image, 1: nearest edge pixel
    int32_t aligned;        // input rows 4-byte aligned and output rows 16-byte aligned
    int32_t pad_;
};

struct ZeroArgs {
    uint32_t *ptr[2 * kMaxStack + 1];
    int64_t words[2 * kMaxStack + 1];
    int32_t count;
};

// Timing events for one launch of kernel `name`: both null unless profiling
// is on for that name (mtb_profile_begin).  The launch carries them in its
// own dispatch, so timing adds no work to the stream between kernels.
struct ProfEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
ProfEvents prof_take(const char *name);
// Files the events of a launch that returned `launched` (or recycles them).
void prof_commit(const char *name, const ProfEvents &ev, hipError_t launched);

// Launches k<<<grid, block, 0, s>>>(a), timed when profiling is on.
// Failure injection for tests (mtb_test_fail_launch): true when this launch
// is to fail without being issued.
bool injected_launch_failure();
// Records the shape of the calling thread's last k_pyramid launch (tests).
void note_pyramid_launch(int blocks, int merged);

template <typename A>
hipError_t launch_kernel(const char *name, void (*k)(A), dim3 grid, dim3 block, hipStream_t s, A a)
{
    if (injected_launch_failure())
        return hipErrorLaunchFailure;
    const ProfEvents ev = prof_take(name);
    void *args[] = {&a};
    const hipError_t e = hipExtLaunchKernel((const void *)k, grid, block, args, 0, s, ev.start, ev.stop, 0);
    prof_commit(name, ev, e);
    return e;
}

// Launch shapes a tuner may change (results never depend on them): k_pyramid
// workgroups as a percentage of one resident round and the tiles of a row a
// workgroup takes at a time (2^pyr_group_log2); k_bitmaps workgroups as a
// percentage of one resident round and wavefronts per workgroup; how many of
// the coarsest levels are searched over exhaustive windows (-1: the rule);
// and per fine level the rows per stream (0: the rule that keeps the grid
// within one resident round) and the lanes per row stream (log2, 3 .. 6; 0:
// the rule that pads rows least).
constexpr int kRowsStep = 4;   // rows per stream come in multiples of this
constexpr int kRowsMax = 64;
struct LaunchTune {
    int32_t pyr_pct = 100;
    int32_t pyr_group_log2 = 0;
    int32_t bm_pct = 100;
    int32_t bm_waves = 4;
    int32_t coarse = -1;
    int32_t small = -1;   // one-workgroup search where a pair fits LDS: -1 or 1 yes, 0 never
    int32_t l1 = -1;      // level 1's bitmaps from level 0's gray: -1 rule, 0 never, 1 always
    int32_t rows[kMaxLevels] = {};
    int32_t cw[kMaxLevels] = {};
};

// Launch helpers (mtb_kernels.hip).  Each returns the hipError_t of its launches.
hipError_t launch_zero(const ZeroArgs &a, hipStream_t s);
hipError_t launch_pyramid(const PyramidArgs &a, int device_cus, hipStream_t s, int slots_pct = 100,
                          int group_log2 = 0);
hipError_t launch_bitmaps(const BitmapArgs &a, int device_cus, hipStream_t s, int blocks_pct = 100, int waves = 4);
hipError_t launch_apply(const ApplyArgs &a, int device_cus, hipStream_t s);
// The byte-map comparison path: T/E as 255/0 bytes, and the search over them.
hipError_t launch_bytemaps(const BitmapArgs &a, int device_cus, hipStream_t s);
hipError_t launch_search_bytes(SearchArgs a, int device_cus, hipStream_t s);
// Turns the pairwise shifts of a chained stack (image i against its neighbour
// towards ref) into shifts against ref, in place.
hipError_t launch_chain(int32_t *d_shifts, int n, int ref, hipStream_t s);
// d_flag[0] = 1 if two of the four shifts differ by more than tol along an axis.
hipError_t launch_quadrant_flag(const int32_t *d_shifts, int32_t tol, int32_t *d_flag, hipStream_t s);
// Searches every level of every pair and writes a.out; a.state and *a.done
// must be zero unless small_search_used(a.g, t).
// Levels L-1 .. L-coarse_level_count(g, npairs) are searched exhaustively;
// the others are the fine levels.
int coarse_level_count(const Geometry &g, int npairs);
// Rows per stream launch_search uses at fine level l without a tuned value
// (for a stream width cw_log2, 0: the rule).
int search_rows_rule(const Geometry &g, int l, int npairs, int device_cus, int cw_log2 = 0);
int search_row_blocks(const Geometry &g, int l, int rows, int cw_log2 = 0);
// Coarse levels a search runs with shape t (null: the rule).
int coarse_levels_used(const Geometry &g, int npairs, const LaunchTune *t);
// A pair whose two bitmap pyramids (every plane, as laid out in the bitmaps
// buffer) fit kSmallLdsBytes is searched by one workgroup that holds both in
// LDS and runs every level (k_search_small): one launch, no search state.
constexpr int64_t kSmallLdsBytes = 144 * 1024;
bool small_search_fits(const Geometry &g);
// Whether launch_search takes the one-workgroup search with shape t (null: the rule).
bool small_search_used(const Geometry &g, const LaunchTune *t);
// t: the launch shape (rows and lanes per stream per level, coarse levels), or null for the rules.
hipError_t launch_search(SearchArgs a, int device_cus, hipStream_t s, const LaunchTune *t = nullptr);

}  // namespace mtb
