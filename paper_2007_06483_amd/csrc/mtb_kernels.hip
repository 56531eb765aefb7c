// mtb_kernels.hip -- gfx950 kernels for MTB translational alignment.
//
// Pass 1  k_pyramid         RGB -> gray levels 0..6 of 64x256 tiles + LDS histograms
//         k_pyramid_coarse  levels 7.. from level 6 (one workgroup per image)
// Pass 2  k_bitmaps         gray -> lower median per level, packed T/E words
// Search  k_search_coarse   small levels, one workgroup per pair, all in one launch
//         k_search_fine     one launch per large level, grid over (units, pairs);
//                           the last workgroup of the level-0 launch writes the results
//
// The arithmetic is integer throughout; reductions are integer adds, so the
// results do not depend on the order in which workgroups finish.

#include <atomic>

#include "mtb_internal.h"

namespace mtb {

namespace {

constexpr int kWave = 64;
// Fine search: rows per batch and batches in flight per stream (rows per
// stream is a multiple of their product).
constexpr int kSearchBatch = 1;
constexpr int kSearchDepth = 4;

// Index of the calling wavefront in its workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// 64-bit mask of the lanes whose predicate holds (the predicate stays a lane mask).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// ---------------------------------------------------------------- zero fill

__global__ __launch_bounds__(256) void k_zero(ZeroArgs a)
{
    const int r = blockIdx.y;
    uint32_t *p = a.ptr[r];
    const int64_t n = a.words[r];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------- pass 1

// Ward's integer gray weights; they sum to 256 so the result fits a byte.
__device__ __forceinline__ uint32_t gray3(uint32_t r, uint32_t g, uint32_t b)
{
    return (54u * r + 183u * g + 19u * b) >> 8;
}

// Gray of 4 interleaved RGB pixels held in 3 little-endian dwords
// (R0 G0 B0 R1 | G1 B1 R2 G2 | B2 R3 G3 B3), with byte dot products.
__device__ __forceinline__ void gray4(uint32_t a, uint32_t b, uint32_t c, uint32_t *g)
{
    g[0] = __builtin_amdgcn_udot4(a, 0x0013B736u, 0u, false) >> 8;
    g[1] = __builtin_amdgcn_udot4(b, 0x000013B7u, __builtin_amdgcn_udot4(a, 0x36000000u, 0u, false), false) >> 8;
    g[2] = __builtin_amdgcn_udot4(c, 0x00000013u, __builtin_amdgcn_udot4(b, 0xB7360000u, 0u, false), false) >> 8;
    g[3] = __builtin_amdgcn_udot4(c, 0x13B73600u, 0u, false) >> 8;
}

__device__ __forceinline__ uint32_t pack4(const uint32_t *v)
{
    return v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
}

// Loads and stores of words that several workgroups (on different XCDs) exchange
// within one launch: agent-scope atomics, performed at the coherence point.
__device__ __forceinline__ uint32_t load_shared(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_shared(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Level-0 histogram privatisation: kH0Copies copies per wave; copies kHStride
// (odd) words apart, so that equal values from lanes of different copies fall
// into different LDS banks.  Atomics to one address serialise, and nearby
// pixels are often equal, so the lanes sharing a copy should hold pixels far
// apart: lane (bx, by) (pixels at x = 16 bx + c, y = 4 by + r) adds into copy
// (bx + 2 by) mod 8, whose lanes are at least 32 columns or 8 rows apart.
constexpr int kH0Copies = 8;
constexpr int kHStride = 257;

// Clang vector type, the operand type the nontemporal builtins accept.
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));

// Loads one lane's 4 rows x 48 bytes (16 pixels) of RGB with 16-byte loads;
// rows at or below H read as zero.
__device__ __forceinline__ void load_rgb16(const uint8_t *rgb, int64_t stride, int x0, int y0, int H,
                                           uint4 (&q)[4][3])
{
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        if (y0 + rr < H) {
            const uint4 *p = (const uint4 *)(rgb + (int64_t)(y0 + rr) * stride + 3 * (int64_t)x0);
            q[rr][0] = p[0];
            q[rr][1] = p[1];
            q[rr][2] = p[2];
        } else {
            q[rr][0] = q[rr][1] = q[rr][2] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
}

// Tiles whose levels 5 and 6 wait in an LDS ring; the ring is drained by the
// whole workgroup after one barrier, instead of one barrier per tile.
constexpr int kDefer = 8;

// Workgroup tile: kTileH = 64 rows x kTileW = 256 columns of level 0.  Wave w
// owns rows 16w .. 16w+15; lane (bx = lane & 15, by = lane >> 4) owns the
// 4-row x 16-column block at (X0 + 16 bx, Y0 + 16 w + 4 by).  Levels 1 and 2
// stay inside the lane, levels 3 and 4 combine lanes of the wave with
// shuffles, levels 5 and 6 combine the four waves through LDS: a tile's 4 x 16
// level-4 pixels are parked in a ring of kDefer tiles, and a full ring is
// turned into levels 5 and 6 by all 256 threads at once.  Each lane
// reads 4 x 48 bytes of RGB per tile (a row of 16 lanes covers 768
// contiguous bytes), and with 16-byte aligned rows the next tile's RGB is
// loaded while the current one is processed.
__global__ __launch_bounds__(256) void k_pyramid(PyramidArgs a)
{
    __shared__ uint32_t hist0[4 * kH0Copies * kHStride];  // level 0, per wave and lane group
    __shared__ uint32_t hist1[4][256];                    // level 1, per wave
    __shared__ uint32_t histc[kFused - 2][256];           // levels 2 .. 6, whole workgroup
    __shared__ uint32_t lvl4[2][kDefer][4][16];           // level-4 pixels of deferred tiles, two rings
    __shared__ int2 ring_pos[2][kDefer];                  // level-0 origin of each deferred tile
    __shared__ int s_merge;                               // this workgroup merges the image's copies

    const int tid = threadIdx.x;
    const int wave = wave_id();
    const int lane = tid & 63;
    const int bx = lane & 15, by = lane >> 4;
    const Geometry &g = a.g;
    const int fused = g.L < kFused ? g.L : kFused;
    uint32_t *h0 = hist0 + (wave * kH0Copies + ((bx + 2 * by) & (kH0Copies - 1))) * kHStride;

    for (int i = tid; i < 4 * kH0Copies * kHStride; i += 256)
        hist0[i] = 0u;
    for (int i = tid; i < 4 * 256; i += 256)
        (&hist1[0][0])[i] = 0u;
    for (int i = tid; i < (kFused - 2) * 256; i += 256)
        (&histc[0][0])[i] = 0u;
    __syncthreads();

    const int64_t per_image = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t total = per_image * a.n;
    // XCD-aware schedule.  Workgroups are dealt to the XCDs in turn, so
    // workgroup b runs on XCD b % kXcds, and each XCD takes a contiguous share
    // of the tiles (image-major, then row bands, then columns).  Its slots walk
    // that share in step, slot s taking tiles s, s + slots, ...: neighbouring
    // tiles of a row band are read at the same time on the same XCD, so the
    // cache line two of them share is fetched from HBM once.
    const int slot = blockIdx.x / kXcds, slots = gridDim.x / kXcds;
    const int64_t xb = (int64_t)(blockIdx.x % kXcds) * a.xcd_tiles;
    const int64_t t0 = xb + ((int64_t)slot << a.group_log2);
    const int64_t t1 = xb + a.xcd_tiles < total ? xb + a.xcd_tiles : total;
    // The share is walked in groups of 2^group_log2 consecutive tiles (one
    // launch-shape knob): slot s takes groups s, s + slots, ..., each group's
    // tiles one after another.
    const int64_t gmask = ((int64_t)1 << a.group_log2) - 1;
    auto next_tile = [&](int64_t t) -> int64_t {
        const int64_t r = t - xb;
        if ((r & gmask) != gmask)
            return t + 1;
        return xb + (((r >> a.group_log2) + slots) << a.group_log2);
    };

    // Levels 5 and 6 of the `count` tiles parked in ring `bank` (image img).
    // Call after a barrier that follows the tiles' level-4 writes; thread
    // tid takes pixel tid % 20 of ring entry tid / 20 (16 level-5 pixels in
    // 2 rows of 8, then 4 level-6 pixels).
    auto drain = [&](int img, int bank, int count) {
        const int k = tid / 20, r = tid - 20 * (tid / 20);
        if (k >= count)
            return;
        const uint32_t(*qq)[16] = lvl4[bank][k];
        const int2 o = ring_pos[bank][k];
        uint8_t *pyr = a.pyr[img];
        if (r < 16) {
            const int i5 = r >> 3, j5 = r & 7;
            const uint32_t u5 = (qq[2 * i5][2 * j5] + qq[2 * i5][2 * j5 + 1] + qq[2 * i5 + 1][2 * j5] +
                                 qq[2 * i5 + 1][2 * j5 + 1]) >> 2;
            const LevelGeom &l5 = g.lv[5];
            const int x5 = (o.x >> 5) + j5, y5 = (o.y >> 5) + i5;
            if (y5 < l5.h && x5 < l5.w) {
                pyr[l5.gray_off + (int64_t)y5 * l5.gray_pitch + x5] = (uint8_t)u5;
                atomicAdd(&histc[3][u5], 1u);
            }
        } else if (fused > 6) {
            const int j6 = r - 16;
            uint32_t s6 = 0;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 2 * j6; j < 2 * j6 + 2; ++j)
                    s6 += (qq[2 * i][2 * j] + qq[2 * i][2 * j + 1] + qq[2 * i + 1][2 * j] +
                           qq[2 * i + 1][2 * j + 1]) >> 2;
            const uint32_t u6 = s6 >> 2;
            const LevelGeom &l6 = g.lv[6];
            const int x6 = (o.x >> 6) + j6, y6 = o.y >> 6;
            if (y6 < l6.h && x6 < l6.w) {
                pyr[l6.gray_off + (int64_t)y6 * l6.gray_pitch + x6] = (uint8_t)u6;
                atomicAdd(&histc[4][u6], 1u);
            }
        }
    };
    int bank = 0, parked = 0;

    // Tiles of image img in XCD x's share of the tiles.
    auto xcd_tiles_of = [&](int x, int img) -> int64_t {
        const int64_t ib = (int64_t)img * per_image, ie = ib + per_image;
        int64_t b = (int64_t)x * a.xcd_tiles, e = b + a.xcd_tiles < total ? b + a.xcd_tiles : total;
        b = b > ib ? b : ib;
        e = e < ie ? e : ie;
        return e > b ? e - b : 0;
    };

    // Adds the workgroup's histograms of image img (from `tiles` of its tiles)
    // into the image's histogram, or with a.merge into its XCD's copy in the
    // merge scratch, summed into the histogram by the workgroup that adds the
    // image's last tiles.  When hundreds of workgroups of an image flush at
    // the same moment (a few tiles each), their atomics on the histogram's
    // few cache lines queue behind each other; the copies divide that queue
    // by the XCD count, at the price of a ticket round trip per flush.  The
    // tickets follow the ordering of last_workgroup: agent-scope atomics
    // only, each thread's own operations acknowledged before the workgroup
    // takes its ticket.  The tile ticket of each XCD counts tiles; the
    // workgroup that completes its XCD's tiles of the image takes a ticket
    // among the XCDs holding tiles of the image, and the last of those merges.
    auto flush = [&](int img, int tiles) {
        __syncthreads();
        if (parked > 0) {
            drain(img, bank, parked);
            parked = 0;
            __syncthreads();
        }
        const int xcd = blockIdx.x % kXcds;
        uint32_t *merge = (uint32_t *)(a.pyr[img] + g.hmerge_off);
        uint32_t *gh = a.merge ? merge + xcd * kFused * 256 : (uint32_t *)(a.pyr[img] + g.hist_off);
        for (int l = 0; l < fused; ++l) {
            uint32_t s = 0;
            if (l == 0) {
                for (int c = 0; c < 4 * kH0Copies; ++c) {
                    s += hist0[c * kHStride + tid];
                    hist0[c * kHStride + tid] = 0u;
                }
            } else if (l == 1) {
                s = hist1[0][tid] + hist1[1][tid] + hist1[2][tid] + hist1[3][tid];
                hist1[0][tid] = hist1[1][tid] = hist1[2][tid] = hist1[3][tid] = 0u;
            } else {
                s = histc[l - 2][tid];
                histc[l - 2][tid] = 0u;
            }
            if (s)
                atomicAdd(gh + l * 256 + tid, s);
        }
        if (!a.merge) {
            __syncthreads();
            return;
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            uint32_t *tickets = merge + kXcds * kFused * 256;
            s_merge = 0;
            if ((int64_t)atomicAdd(tickets + xcd, (uint32_t)tiles) + tiles == xcd_tiles_of(xcd, img)) {
                uint32_t holders = 0;
                for (int x = 0; x < kXcds; ++x)
                    holders += xcd_tiles_of(x, img) > 0;
                s_merge = atomicAdd(tickets + kXcds, 1u) + 1 == holders;
            }
        }
        __syncthreads();
        if (s_merge) {
            uint32_t *hist = (uint32_t *)(a.pyr[img] + g.hist_off);
            for (int l = 0; l < fused; ++l) {
                uint32_t v = 0;
                for (int x = 0; x < kXcds; ++x)
                    v += load_shared(merge + (x * kFused + l) * 256 + tid);
                hist[l * 256 + tid] = v;
            }
        }
        __syncthreads();
    };

    // Tile t -> image and level-0 origin of this lane's block.
    auto locate = [&](int64_t t, int &img, int &X0, int &Y0) {
        img = (int)(t / per_image);
        const int64_t r = t - (int64_t)img * per_image;
        X0 = (int)(r % a.tiles_x) * kTileW;
        Y0 = (int)(r / a.tiles_x) * kTileH;
    };

    const bool fast16 = a.align == 16;
    uint4 q[4][3];
    if (fast16 && t0 < t1) {
        int img, X0, Y0;
        locate(t0, img, X0, Y0);
        const int x0 = X0 + 16 * bx;
        if (x0 + 15 < g.W)
            load_rgb16(a.rgb[img], a.stride, x0, Y0 + 16 * wave + 4 * by, g.H, q);
    }

    int cur = -1, cur_tiles = 0;
    for (int64_t t = t0; t < t1; t = next_tile(t)) {
        int img, X0, Y0;
        locate(t, img, X0, Y0);
        if (img != cur) {
            if (cur >= 0)
                flush(cur, cur_tiles);
            cur = img;
            cur_tiles = 0;
        }
        ++cur_tiles;
        const int x0 = X0 + 16 * bx, y0 = Y0 + 16 * wave + 4 * by;
        const uint8_t *rgb = a.rgb[img];
        uint8_t *pyr = a.pyr[img];
        const bool full = x0 + 15 < g.W;

        // ---- level 0: gray of the 4x16 block
        uint32_t gv[4][16];
        if (fast16 && full) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const uint32_t d[12] = {q[rr][0].x, q[rr][0].y, q[rr][0].z, q[rr][0].w,
                                        q[rr][1].x, q[rr][1].y, q[rr][1].z, q[rr][1].w,
                                        q[rr][2].x, q[rr][2].y, q[rr][2].z, q[rr][2].w};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    gray4(d[3 * k], d[3 * k + 1], d[3 * k + 2], &gv[rr][4 * k]);
            }
        } else if (a.align >= 4 && full) {
            uint32_t d[4][12];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const uint32_t *p = (const uint32_t *)(rgb + (int64_t)(y0 + rr) * a.stride + 3 * (int64_t)x0);
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    d[rr][k] = (y0 + rr < g.H) ? p[k] : 0u;
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    gray4(d[rr][3 * k], d[rr][3 * k + 1], d[rr][3 * k + 2], &gv[rr][4 * k]);
        } else if (full) {
            // Rows at any byte alignment: the whole dwords overlapping the lane's
            // 48 bytes (12, or 13 when the start is not 4-aligned; each holds a
            // byte of the segment, so none reaches into a page the row does not
            // touch), moved into place with v_alignbyte_b32.
            uint32_t d[4][12];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const uint8_t *row = rgb + (int64_t)(y0 + rr) * a.stride + 3 * (int64_t)x0;
                const uint32_t sh = (uint32_t)(uintptr_t)row & 3u;
                const uint32_t *p = (const uint32_t *)((uintptr_t)row - sh);
                uint32_t w[13];
                const bool in = y0 + rr < g.H;
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    w[k] = in ? p[k] : 0u;
                w[12] = in && sh ? p[12] : 0u;
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    d[rr][k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    gray4(d[rr][3 * k], d[rr][3 * k + 1], d[rr][3 * k + 2], &gv[rr][4 * k]);
        } else {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const uint8_t *row = rgb + (int64_t)(y0 + rr) * a.stride + 3 * (int64_t)x0;
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    gv[rr][c] = (y0 + rr < g.H && x0 + c < g.W)
                                    ? gray3(row[3 * c], row[3 * c + 1], row[3 * c + 2])
                                    : 0u;
            }
        }
        // ---- prefetch the next tile's RGB while this one is processed
        if (fast16 && next_tile(t) < t1) {
            int img2, X2, Y2;
            locate(next_tile(t), img2, X2, Y2);
            const int x2 = X2 + 16 * bx;
            if (x2 + 15 < g.W)
                load_rgb16(a.rgb[img2], a.stride, x2, Y2 + 16 * wave + 4 * by, g.H, q);
        }
        {
            const LevelGeom &lv = g.lv[0];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int y = y0 + rr;
                if (y < g.H && x0 < g.W) {
                    // x0 % 16 == 0, x0 < W <= pitch, pitch % 64 == 0: 16 bytes inside the row.
                    // Streaming (nontemporal) store: level 0 is read again only by the
                    // next kernel, and keeping it out of L2 speeds up the RGB stream.
                    U32x4 v;
                    v.x = pack4(&gv[rr][0]);
                    v.y = pack4(&gv[rr][4]);
                    v.z = pack4(&gv[rr][8]);
                    v.w = pack4(&gv[rr][12]);
                    __builtin_nontemporal_store(v, (U32x4 *)(pyr + lv.gray_off + (int64_t)y * lv.gray_pitch + x0));
                    if (full) {
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            atomicAdd(&h0[gv[rr][c]], 1u);
                    } else {
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            if (x0 + c < g.W)
                                atomicAdd(&h0[gv[rr][c]], 1u);
                    }
                }
            }
        }
        if (fused > 1) {
            // ---- level 1: 2 x 8 per lane
            uint32_t u1[2][8];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    u1[i][j] = (gv[2 * i][2 * j] + gv[2 * i][2 * j + 1] + gv[2 * i + 1][2 * j] +
                                gv[2 * i + 1][2 * j + 1]) >> 2;
            const LevelGeom &l1 = g.lv[1];
            const int x1 = x0 >> 1, y1 = y0 >> 1;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (y1 + i < l1.h && x1 < l1.w) {
                    if (!a.skip_l1)
                        *(uint2 *)(pyr + l1.gray_off + (int64_t)(y1 + i) * l1.gray_pitch + x1) =
                            make_uint2(pack4(&u1[i][0]), pack4(&u1[i][4]));
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (x1 + j < l1.w)
                            atomicAdd(&hist1[wave][u1[i][j]], 1u);
                }
            }
            if (fused > 2) {
                // ---- level 2: 1 x 4 per lane
                uint32_t u2[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    u2[j] = (u1[0][2 * j] + u1[0][2 * j + 1] + u1[1][2 * j] + u1[1][2 * j + 1]) >> 2;
                const LevelGeom &l2 = g.lv[2];
                const int x2 = x0 >> 2, y2 = y0 >> 2;
                if (y2 < l2.h && x2 < l2.w) {
                    *(uint32_t *)(pyr + l2.gray_off + (int64_t)y2 * l2.gray_pitch + x2) = pack4(u2);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (x2 + j < l2.w)
                            atomicAdd(&histc[0][u2[j]], 1u);
                }
                if (fused > 3) {
                    // ---- level 3: columns inside the lane, rows from lane ^ 16 (by ^ 1)
                    uint32_t u3[2];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        uint32_t s3 = u2[2 * j] + u2[2 * j + 1];
                        s3 += __shfl_xor(s3, 16);
                        u3[j] = s3 >> 2;
                    }
                    const LevelGeom &l3 = g.lv[3];
                    const int x3 = x0 >> 3, y3 = y0 >> 3;
                    if ((by & 1) == 0 && y3 < l3.h && x3 < l3.w) {
                        *(uint16_t *)(pyr + l3.gray_off + (int64_t)y3 * l3.gray_pitch + x3) =
                            (uint16_t)(u3[0] | (u3[1] << 8));
                        atomicAdd(&histc[1][u3[0]], 1u);
                        if (x3 + 1 < l3.w)
                            atomicAdd(&histc[1][u3[1]], 1u);
                    }
                    if (fused > 4) {
                        // ---- level 4: rows from lane ^ 32 (by ^ 2); owners are lanes 0..15
                        uint32_t s4 = u3[0] + u3[1];
                        s4 += __shfl_xor(s4, 32);
                        const uint32_t u4 = s4 >> 2;
                        const LevelGeom &l4 = g.lv[4];
                        const int x4 = x0 >> 4, y4 = y0 >> 4;
                        if (by == 0 && y4 < l4.h && x4 < l4.w) {
                            pyr[l4.gray_off + (int64_t)y4 * l4.gray_pitch + x4] = (uint8_t)u4;
                            atomicAdd(&histc[2][u4], 1u);
                        }
                        if (fused > 5) {
                            // ---- levels 5 and 6: park the tile's 4 x 16 level-4 pixels
                            // (row = wave, column = bx); a full ring is drained.
                            if (by == 0)
                                lvl4[bank][parked][wave][bx] = u4;
                            if (tid == 0)
                                ring_pos[bank][parked] = make_int2(X0, Y0);
                            if (++parked == kDefer) {
                                __syncthreads();
                                drain(img, bank, kDefer);
                                bank ^= 1;
                                parked = 0;
                            }
                        }
                    }
                }
            }
        }
    }
    if (cur >= 0)
        flush(cur, cur_tiles);
}

// Levels kFused .. L-1, each the floor 2x2 mean of the level below; one
// workgroup per image, levels one after another.
__global__ __launch_bounds__(256) void k_pyramid_coarse(CoarsePyramidArgs a)
{
    __shared__ uint32_t hist[256];
    const int img = blockIdx.x;
    const Geometry &g = a.g;
    uint8_t *pyr = a.pyr[img];
    for (int l = kFused; l < g.L; ++l) {
        hist[threadIdx.x] = 0u;
        __syncthreads();
        const LevelGeom &lo = g.lv[l], &hi = g.lv[l - 1];
        const int np = lo.w * lo.h;
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            const int x = i % lo.w, y = i / lo.w;
            const uint8_t *s0 = pyr + hi.gray_off + (int64_t)(2 * y) * hi.gray_pitch + 2 * x;
            const uint8_t *s1 = s0 + hi.gray_pitch;
            const uint32_t u = ((uint32_t)s0[0] + s0[1] + s1[0] + s1[1]) >> 2;
            pyr[lo.gray_off + (int64_t)y * lo.gray_pitch + x] = (uint8_t)u;
            atomicAdd(&hist[u], 1u);
        }
        __syncthreads();
        ((uint32_t *)(pyr + g.hist_off))[l * 256 + threadIdx.x] = hist[threadIdx.x];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- pass 2

// A 256-bin histogram as one wavefront holds it: bins 4i .. 4i + 3 in lane i.
__device__ __forceinline__ uint4 wave_hist(const uint32_t *hist)
{
    return *(const uint4 *)(hist + 4 * (threadIdx.x & 63));
}

// Lower median of a 256-bin histogram (as wave_hist loads it) holding npix
// pixels, computed by one wavefront: smallest v whose cumulative count
// reaches ceil(npix / 2).
__device__ uint32_t wave_median_of(const uint4 h, uint32_t npix)
{
    const int lane = threadIdx.x & 63;
    const uint32_t s = h.x + h.y + h.z + h.w;
    uint32_t incl = s;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d);
        if (lane >= d)
            incl += o;
    }
    const uint32_t need = (npix + 1u) >> 1;
    const uint64_t hit = ballot(incl >= need);
    const int f = __ffsll((unsigned long long)hit) - 1;
    uint32_t v = 0;
    if (lane == f) {
        uint32_t c = incl - s;
        v = 4 * lane + 3;
        if ((c += h.x) >= need)
            v = 4 * lane;
        else if ((c += h.y) >= need)
            v = 4 * lane + 1;
        else if ((c += h.z) >= need)
            v = 4 * lane + 2;
    }
    return __builtin_amdgcn_readfirstlane(__shfl(v, f < 0 ? 0 : f));
}

__device__ __forceinline__ uint32_t wave_median(const uint32_t *hist, uint32_t npix)
{
    return wave_median_of(wave_hist(hist), npix);
}


struct ChunkPos {
    int img, level, w0, cnt;
};

// Chunk c of a walk over levels l0 .. L-1 of every image (per_image chunks
// each).
__device__ __forceinline__ ChunkPos chunk_pos(const BitmapArgs &a, int64_t c, int64_t per_image, int l0)
{
    ChunkPos p;
    p.img = (int)(c / per_image);
    const int64_t cc = c - (int64_t)p.img * per_image + a.chunk_start[l0];
    int l = l0;
    while (cc >= a.chunk_start[l + 1])
        ++l;
    p.level = l;
    p.w0 = (int)(cc - a.chunk_start[l]) * kChunkWords;
    const int nwords = a.g.lv[l].h * a.g.lv[l].wpr;
    p.cnt = nwords - p.w0 < kChunkWords ? nwords - p.w0 : kChunkWords;
    return p;
}

// The chunk after p in a walk over levels l0 .. L-1, and col0 = p.w0 mod wpr
// of its level, without divisions (every level holds at least one word).
__device__ __forceinline__ void next_chunk(const BitmapArgs &a, ChunkPos &p, int &col0, int l0)
{
    const LevelGeom *lv = &a.g.lv[p.level];
    p.w0 += kChunkWords;
    int nwords = lv->h * lv->wpr;
    if (p.w0 >= nwords) {
        p.w0 = 0;
        col0 = 0;
        if (++p.level == a.g.L) {
            p.level = l0;
            ++p.img;
        }
        lv = &a.g.lv[p.level];
        nwords = lv->h * lv->wpr;
    } else if (lv->wpr >= kChunkWords) {
        col0 += kChunkWords;
        if (col0 >= lv->wpr)
            col0 -= lv->wpr;
    } else {
        col0 = (col0 + kChunkWords) % lv->wpr;
    }
    p.cnt = nwords - p.w0 < kChunkWords ? nwords - p.w0 : kChunkWords;
}

// Lane i's 32 pixels of a chunk: bytes [32 i, 32 i + 32), zero past the chunk.
__device__ __forceinline__ void load_chunk(const BitmapArgs &a, const ChunkPos &p, int lane, uint4 &v0, uint4 &v1)
{
    const uint8_t *src = a.pyr[p.img] + a.g.lv[p.level].gray_off + (int64_t)p.w0 * 64 + lane * 32;
    const bool in = lane < 2 * p.cnt;
    v0 = in ? ((const uint4 *)src)[0] : make_uint4(0u, 0u, 0u, 0u);
    v1 = in ? ((const uint4 *)src)[1] : make_uint4(0u, 0u, 0u, 0u);
}

// Byte-wise x >= y for a uniform threshold y in [0, 255], four bytes at once;
// the answer is bit 7 of each byte (the other bits are undefined).  With
// xh = x | 0x80808080 and low = (y & 0x7f) * 0x01010101, each byte of xh - low
// is 0x80 + (x & 0x7f) - (y & 0x7f), in [1, 255], so no byte borrows from the
// next and its bit 7 is [x & 0x7f >= y & 0x7f].  Bit 7 of x and y decides the
// rest: y < 128 (sel all ones) gives x7 | d7, y >= 128 (sel 0) gives x7 & d7.
struct ByteGe {
    uint32_t low, sel;
};
__device__ __forceinline__ ByteGe byte_ge(uint32_t y)
{
    return ByteGe{(y & 0x7fu) * 0x01010101u, y < 128u ? ~0u : 0u};
}
__device__ __forceinline__ uint32_t ge_bytes(uint32_t x, uint32_t xh, ByteGe c)
{
    const uint32_t d = xh - c.low;
    return (x & d) | (c.sel & (x | d));
}

// Eight dwords d[k] holding pixels 4k .. 4k+3 (byte b = pixel 4k + b) are
// transposed so that t[k] holds pixels k, k+8, k+16, k+24 (byte b = pixel 8b + k).
// v_perm_b32 (__builtin_amdgcn_perm(hi, lo, sel)): selector byte values 0-3
// pick bytes of lo, 4-7 bytes of hi.
__device__ __forceinline__ void transpose8(const uint32_t *d, uint32_t *t)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // h = 0: dwords 0,2,4,6 -> t[0..3]; h = 1: 1,3,5,7 -> t[4..7]
        const uint32_t A = __builtin_amdgcn_perm(d[2 + h], d[0 + h], 0x05010400u);  // d0.b0 d2.b0 d0.b1 d2.b1
        const uint32_t B = __builtin_amdgcn_perm(d[2 + h], d[0 + h], 0x07030602u);  // d0.b2 d2.b2 d0.b3 d2.b3
        const uint32_t C = __builtin_amdgcn_perm(d[6 + h], d[4 + h], 0x05010400u);  // d4.b0 d6.b0 d4.b1 d6.b1
        const uint32_t D = __builtin_amdgcn_perm(d[6 + h], d[4 + h], 0x07030602u);  // d4.b2 d6.b2 d4.b3 d6.b3
        t[4 * h + 0] = __builtin_amdgcn_perm(C, A, 0x05040100u);
        t[4 * h + 1] = __builtin_amdgcn_perm(C, A, 0x07060302u);
        t[4 * h + 2] = __builtin_amdgcn_perm(D, B, 0x05040100u);
        t[4 * h + 3] = __builtin_amdgcn_perm(D, B, 0x07060302u);
    }
}

// The three thresholds of a level, T: m + 1, E: m + X + 1 and max(m - X, 0),
// as byte-wise comparison constants; keep_* clear a threshold above 255.
struct Thresholds {
    uint32_t low_t, low_hi, low_lo, keep_t, keep_hi;
    int nlow;  // how many thresholds are below 128 (lo <= t <= hi, so a prefix)
};
__device__ __forceinline__ Thresholds thresholds(uint32_t m, uint32_t X)
{
    const uint32_t yt = m + 1u, yhi = m + X + 1u, ylo = m > X ? m - X : 0u;
    Thresholds c;
    c.low_t = (yt & 0x7fu) * 0x01010101u;
    c.low_hi = (yhi & 0x7fu) * 0x01010101u;
    c.low_lo = (ylo & 0x7fu) * 0x01010101u;
    c.keep_t = yt < 256u ? ~0u : 0u;
    c.keep_hi = yhi < 256u ? ~0u : 0u;
    c.nlow = (ylo < 128u) + (yt < 128u) + (yhi < 128u);
    return c;
}

// T and E bits of a lane's 32 transposed pixels (byte b of t[k] = pixel 8b + k)
// with ge_bytes specialised on which thresholds are below 128: x >= y is bit 7
// of x | d for y < 128 and of x & d otherwise (d = (x | 0x80808080) - low).
// Bit 7 of byte b of each answer moves to bit 8b + k of the word.
template <bool kLowT, bool kLowHi, bool kLowLo>
__device__ __forceinline__ void te_bits(const uint32_t (&t)[8], const Thresholds &c, uint32_t &tw, uint32_t &ew)
{
    tw = 0u;
    ew = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t x = t[k], xh = x | 0x80808080u;
        const uint32_t dt = xh - c.low_t, dhi = xh - c.low_hi, dlo = xh - c.low_lo;
        const uint32_t gt = kLowT ? (x | dt) : (x & dt);
        const uint32_t ghi = kLowHi ? (x | dhi) : (x & dhi);
        const uint32_t glo = kLowLo ? (x | dlo) : (x & dlo);
        const uint32_t rt = gt & c.keep_t;
        const uint32_t re = (ghi & c.keep_hi) | ~glo;
        tw |= (rt >> (7 - k)) & (0x01010101u << k);
        ew |= (re >> (7 - k)) & (0x01010101u << k);
    }
}

// Each wavefront walks a contiguous run of chunks of kChunkWords = 32
// consecutive 64-pixel words of one level (the next chunk's loads are issued
// before the current one is processed).  Lane i takes the chunk's bytes
// [32 i, 32 i + 32), i.e. half-word i of the chunk, and forms its 32 T and E
// bits in registers: four pixels per dword compared at once (ByteGe), after a
// byte transpose that lets the per-byte answers be gathered into bit order
// with one shift and one and-or per dword.  Lane i then stores dword i of the
// chunk's T words and of its E words.  This walks chunks c0 .. c1 - 1 of
// levels l0 .. L-1 of every image (per_image chunks each).
__device__ __forceinline__ void walk_chunks(const BitmapArgs &a, int64_t c0, int64_t c1, int64_t per_image, int l0,
                                            int lane)
{
    const Geometry &g = a.g;
    const uint32_t X = (uint32_t)a.exclude;

    int cur_img = -1, cur_l = -1;
    uint32_t m = 0;
    Thresholds th = thresholds(0u, X);
    ChunkPos p = chunk_pos(a, c0, per_image, l0);
    int col0 = p.w0 % g.lv[p.level].wpr;
    uint4 v0, v1;
    load_chunk(a, p, lane, v0, v1);
    for (int64_t c = c0; c < c1; ++c) {
        const ChunkPos cp = p;
        const int ccol0 = col0;
        const LevelGeom &lv = g.lv[cp.level];
        if (cp.img != cur_img || cp.level != cur_l) {
            m = wave_median((const uint32_t *)(a.pyr[cp.img] + g.hist_off) + 256 * cp.level,
                            (uint32_t)(lv.w * lv.h));
            cur_img = cp.img;
            cur_l = cp.level;
            // T = [g >= m + 1]; E = [g >= m + X + 1] | ~[g >= max(m - X, 0)].
            th = thresholds(m, X);
        }
        if (cp.w0 == 0 && lane == 0)
            ((int32_t *)(a.bm[cp.img] + g.med_off))[cp.level] = (int32_t)m;

        const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        if (c + 1 < c1) {
            next_chunk(a, p, col0, l0);
            load_chunk(a, p, lane, v0, v1);
        }
        uint32_t t[8];
        transpose8(d, t);
        uint32_t tw, ew;
        switch (th.nlow) {
        case 0: te_bits<false, false, false>(t, th, tw, ew); break;
        case 1: te_bits<false, false, true>(t, th, tw, ew); break;
        case 2: te_bits<true, false, true>(t, th, tw, ew); break;
        default: te_bits<true, true, true>(t, th, tw, ew); break;
        }
        // Bits past the level width are zero: lane i holds half-word i % 2 of
        // word w0 + i / 2, whose pixels start at column 64 * ((w0 + i / 2) mod wpr).
        int col = ccol0 + (lane >> 1);
        if (lv.wpr >= kChunkWords)
            col = col >= lv.wpr ? col - lv.wpr : col;
        else
            col = col % lv.wpr;
        const int nbits = lv.w - 64 * col - 32 * (lane & 1);
        const uint32_t keep = nbits >= 32 ? ~0u : (nbits <= 0 ? 0u : (1u << nbits) - 1u);
        if (lane < 2 * cp.cnt) {
            ((uint32_t *)(a.bm[cp.img] + lv.tb_off))[2 * (int64_t)cp.w0 + lane] = tw & keep;
            ((uint32_t *)(a.bm[cp.img] + lv.eb_off))[2 * (int64_t)cp.w0 + lane] = ew & keep;
        }
    }
}

// T and E answers of four pixels (byte b = pixel b) in bit 7 of each byte,
// the case of te_bits picked at run time.
__device__ __forceinline__ void te4(uint32_t x, const Thresholds &c, uint32_t &rt, uint32_t &re)
{
    const uint32_t xh = x | 0x80808080u;
    const uint32_t dt = xh - c.low_t, dhi = xh - c.low_hi, dlo = xh - c.low_lo;
    const uint32_t sl = c.nlow >= 1 ? ~0u : 0u, st = c.nlow >= 2 ? ~0u : 0u, sh = c.nlow >= 3 ? ~0u : 0u;
    const uint32_t glo = (x & dlo) | (sl & (x | dlo));
    const uint32_t gt = (x & dt) | (st & (x | dt));
    const uint32_t ghi = (x & dhi) | (sh & (x | dhi));
    rt = gt & c.keep_t;
    re = (ghi & c.keep_hi) | ~glo;
}

// Bit 7 of byte b of r0 moved to bit b and bit 7 of byte b of r1 to bit 4 + b.
// After the shifts byte b holds r0's bit at 8b and r1's at 8b + 4; the
// product takes them to 24 + b and 28 + b (0x01020408 = 2^24 + 2^17 + 2^10 +
// 2^3), and every other partial product lands below bit 24 or above bit 31,
// each on a bit of its own, so nothing carries into bits 24..31.
__device__ __forceinline__ uint32_t bits8(uint32_t r0, uint32_t r1)
{
    const uint32_t u = ((r0 >> 7) & 0x01010101u) | ((r1 >> 3) & 0x10101010u);
    return (u * 0x01020408u) >> 24;
}

// The 8 level-1 pixels below a lane's 2 x 16 level-0 pixels of a pair unit
// (d[0..3] row 2j, d[4..7] row 2j + 1, byte b of d[k] = pixel 4k + b): the
// floor means of the 2x2 blocks, pixels 4h .. 4h + 3 in bytes 0..3 of g1[h].
// Per dword pair: 16-bit sums of pixels (4k, 4k + 1) and (4k + 2, 4k + 3) of
// both rows (bytes 1 and 3 moved down by a v_perm_b32 whose selector 0x0c
// yields zero bytes), a quarter of each in byte 0 and byte 2 (sums are at
// most 1020, so the shift leaves each in its own byte), then bytes 0 and 2
// of two such dwords gathered by one more v_perm_b32.
__device__ __forceinline__ void level1_gray(const uint32_t (&d)[8], uint32_t (&g1)[2])
{
    uint32_t q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t a = d[k], b = d[k + 4];
        const uint32_t sum = (a & 0x00ff00ffu) + __builtin_amdgcn_perm(0u, a, 0x0c030c01u) + (b & 0x00ff00ffu) +
                             __builtin_amdgcn_perm(0u, b, 0x0c030c01u);
        q[k] = sum >> 2;
    }
    g1[0] = __builtin_amdgcn_perm(q[1], q[0], 0x06040200u);
    g1[1] = __builtin_amdgcn_perm(q[3], q[2], 0x06040200u);
}

// Segments of kPairWords words in a level-0 row.
__device__ __forceinline__ int pair_segments(const Geometry &g) { return (g.lv[0].wpr + kPairWords - 1) / kPairWords; }

// Lane `lane`'s gray bytes of pair unit (img, j, s): its 16 pixels of row 2j
// (v0) and of row 2j + 1 (v1), columns 64 kPairWords s + 16 lane ..  The
// loads never branch: a lane past the row's words reads the row's last 16
// bytes and a missing row 2j + 1 (odd height) reads row 2j again; pair_unit
// stores nothing from either (no level-0 bits past the row, zero level-1
// bits past level 1's width, no level-1 row without row 2j + 1).
__device__ __forceinline__ void load_unit(const BitmapArgs &a, int img, int j, int s, int lane, uint4 &v0, uint4 &v1)
{
    const LevelGeom &lv = a.g.lv[0];
    const int col = 64 * kPairWords * s + 16 * lane;
    const int colc = col < (int)lv.gray_pitch - 16 ? col : (int)lv.gray_pitch - 16;
    const uint8_t *row = a.pyr[img] + lv.gray_off + (int64_t)(2 * j) * lv.gray_pitch;
    v0 = *(const uint4 *)(row + colc);
    v1 = *(const uint4 *)(row + (2 * j + 1 < lv.h ? lv.gray_pitch : 0) + colc);
}

// Stores pair unit (img, j, s)'s level-0 T and E bits of the lane (tw, ew:
// bits 0..15 its 16 pixels of row 2j, bits 16..31 those of row 2j + 1) and
// the T and E bits of the 8 level-1 pixels g1 below them.  Lanes past a row's
// words store no level-0 bits; their level-1 bits lie past level 1's width
// and are stored as the row's zero padding.
__device__ __forceinline__ void pair_unit(const BitmapArgs &a, int img, int j, int s, int lane,
                                          const uint32_t (&g1)[2], uint32_t tw, uint32_t ew, const Thresholds &th1)
{
    const Geometry &g = a.g;
    const LevelGeom &l0 = g.lv[0], &l1 = g.lv[1];
    uint8_t *bm = a.bm[img];
    const int x = 64 * kPairWords * s + 16 * lane;  // the lane's first level-0 column
    const int nb = g.W - x;
    const uint32_t keep = nb >= 16 ? 0xffffu : (nb <= 0 ? 0u : (1u << nb) - 1u);
    const bool row1 = 2 * j + 1 < l0.h;
    if (kPairWords * s + (lane >> 2) < l0.wpr) {
        const int64_t o = (int64_t)(2 * j) * l0.wpr * 8 + x / 8;  // bytes into row 2j of a plane
        *(uint16_t *)(bm + l0.tb_off + o) = (uint16_t)(tw & keep);
        *(uint16_t *)(bm + l0.eb_off + o) = (uint16_t)(ew & keep);
        if (row1) {
            *(uint16_t *)(bm + l0.tb_off + o + 8 * l0.wpr) = (uint16_t)((tw >> 16) & keep);
            *(uint16_t *)(bm + l0.eb_off + o + 8 * l0.wpr) = (uint16_t)((ew >> 16) & keep);
        }
    }
    if (!row1)
        return;  // level 1 has floor(h / 2) rows
    uint32_t rt0, re0, rt1, re1;
    te4(g1[0], th1, rt0, re0);
    te4(g1[1], th1, rt1, re1);
    const int x1 = x >> 1;
    const int nb1 = l1.w - x1;
    const uint32_t keep1 = nb1 >= 8 ? 0xffu : (nb1 <= 0 ? 0u : (1u << nb1) - 1u);
    if ((x1 >> 6) < l1.wpr) {
        const int64_t o1 = (int64_t)j * l1.wpr * 8 + (x1 >> 3);
        bm[l1.tb_off + o1] = (uint8_t)(bits8(rt0, rt1) & keep1);
        bm[l1.eb_off + o1] = (uint8_t)(bits8(re0, re1) & keep1);
    }
}

// Walks pair units c0 .. c1 - 1 (a.chunk_start[1] per image, images one
// after another).  Each unit is two level-0 rows by kPairWords words: lane i
// takes 16 pixels of each row, the same 32-pixel transpose and compare as a
// chunk give their level-0 T and E bits (row 2j in the low half), and the
// 2x2 means of the same pixels give the 8 level-1 pixels below them, so that
// level 1's gray is never read.
__device__ __forceinline__ void walk_units(const BitmapArgs &a, int64_t c0, int64_t c1, int lane)
{
    const Geometry &g = a.g;
    const uint32_t X = (uint32_t)a.exclude;
    const int64_t units = a.chunk_start[1];
    const int nseg = pair_segments(g);
    int img = (int)(c0 / units);
    int u = (int)(c0 - (int64_t)img * units);
    int j = u / nseg, s = u - j * nseg;
    int cur_img = -1;
    uint32_t m0 = 0, m1 = 0;
    Thresholds th0 = thresholds(0u, X), th1 = th0;
    uint4 v0, v1;
    load_unit(a, img, j, s, lane, v0, v1);
    for (int64_t c = c0; c < c1; ++c) {
        const int ci = img, cj = j, cs = s, cu = u;
        if (ci != cur_img) {
            // Both histograms' loads are issued before either scan.
            const uint32_t *hist = (const uint32_t *)(a.pyr[ci] + g.hist_off);
            const uint4 h0 = wave_hist(hist), h1 = wave_hist(hist + 256);
            m0 = wave_median_of(h0, (uint32_t)(g.lv[0].w * g.lv[0].h));
            m1 = wave_median_of(h1, (uint32_t)(g.lv[1].w * g.lv[1].h));
            th0 = thresholds(m0, X);
            th1 = thresholds(m1, X);
            cur_img = ci;
        }
        if (cu == 0 && lane == 0) {
            ((int32_t *)(a.bm[ci] + g.med_off))[0] = (int32_t)m0;
            ((int32_t *)(a.bm[ci] + g.med_off))[1] = (int32_t)m1;
        }
        const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        if (c + 1 < c1) {
            ++u;
            if (++s == nseg) {
                s = 0;
                ++j;
            }
            if (u == units) {
                u = j = s = 0;
                ++img;
            }
            load_unit(a, img, j, s, lane, v0, v1);
        }
        uint32_t g1[2];
        level1_gray(d, g1);
        uint32_t t[8];
        transpose8(d, t);
        uint32_t tw, ew;
        switch (th0.nlow) {
        case 0: te_bits<false, false, false>(t, th0, tw, ew); break;
        case 1: te_bits<false, false, true>(t, th0, tw, ew); break;
        case 2: te_bits<true, false, true>(t, th0, tw, ew); break;
        default: te_bits<true, true, true>(t, th0, tw, ew); break;
        }
        pair_unit(a, ci, cj, cs, lane, g1, tw, ew, th1);
    }
}

// The bitmaps pass.  Without kPairs every level is walked in chunks.  With
// kPairs (a.pairs; at least two levels) the launch's items are first every
// image's pair units, which yield levels 0 and 1, then every image's chunks
// of levels 2 .. L-1; a wavefront takes a contiguous run of items.
template <int kW, bool kPairs>
__global__ __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(kPairs ? 6 : 1))) void k_bitmaps(BitmapArgs a)
{
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const int64_t per_image = a.chunk_start[a.g.L];
    const int64_t total = per_image * a.n;
    const int64_t nwaves = (int64_t)gridDim.x * kW;
    const int64_t gw = (int64_t)blockIdx.x * kW + wave;
    const int64_t per_wave = (total + nwaves - 1) / nwaves;
    const int64_t c0 = gw * per_wave;
    const int64_t c1 = c0 + per_wave < total ? c0 + per_wave : total;
    if (c0 >= c1)
        return;
    if constexpr (!kPairs) {
        walk_chunks(a, c0, c1, per_image, 0, lane);
    } else {
        const int64_t units = a.chunk_start[1];
        const int64_t nu = units * a.n;
        if (c0 < nu)
            walk_units(a, c0, c1 < nu ? c1 : nu, lane);
        if (c1 > nu)
            walk_chunks(a, (c0 > nu ? c0 : nu) - nu, c1 - nu, per_image - units, 2, lane);
    }
}

// The paper's representation, for comparison: T and E as one byte per pixel
// (255 or 0), rows of gray_pitch bytes, padding bytes 0.  Same chunk walk as
// k_bitmaps; lane i turns bytes [32 i, 32 i + 32) of a chunk into 32 T bytes
// and 32 E bytes with the byte-wise comparisons of ByteGe.
__global__ __launch_bounds__(256) void k_bytemaps(BitmapArgs a)
{
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    const int64_t per_image = a.chunk_start[g.L];
    const int64_t total = per_image * a.n;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int64_t per_wave = (total + nwaves - 1) / nwaves;
    const int64_t c0 = gw * per_wave;
    const int64_t c1 = c0 + per_wave < total ? c0 + per_wave : total;
    if (c0 >= c1)
        return;
    const uint32_t X = (uint32_t)a.exclude;
    int cur_img = -1, cur_l = -1;
    uint32_t m = 0;
    ByteGe ge_t = byte_ge(0), ge_hi = byte_ge(0), ge_lo = byte_ge(0);
    uint32_t keep_t = 0, keep_hi = 0;
    ChunkPos p = chunk_pos(a, c0, per_image, 0);
    uint4 v0, v1;
    load_chunk(a, p, lane, v0, v1);
    for (int64_t c = c0; c < c1; ++c) {
        const ChunkPos cp = p;
        const LevelGeom &lv = g.lv[cp.level];
        if (cp.img != cur_img || cp.level != cur_l) {
            m = wave_median((const uint32_t *)(a.pyr[cp.img] + g.hist_off) + 256 * cp.level,
                            (uint32_t)(lv.w * lv.h));
            cur_img = cp.img;
            cur_l = cp.level;
            ge_t = byte_ge(m + 1u);
            keep_t = m < 255u ? ~0u : 0u;
            ge_hi = byte_ge(m + X + 1u);
            keep_hi = m + X < 255u ? ~0u : 0u;
            ge_lo = byte_ge(m > X ? m - X : 0u);
        }
        if (cp.w0 == 0 && lane == 0)
            ((int32_t *)(a.bm[cp.img] + g.bmed_off))[cp.level] = (int32_t)m;
        const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        if (c + 1 < c1) {
            p = chunk_pos(a, c + 1, per_image, 0);
            load_chunk(a, p, lane, v0, v1);
        }
        // Valid bytes of the lane's 32 (columns below the level width).
        const int nvalid = lv.w - 64 * ((cp.w0 + (lane >> 1)) % lv.wpr) - 32 * (lane & 1);
        uint32_t t[8], e[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t xh = d[k] | 0x80808080u;
            const uint32_t rt = ge_bytes(d[k], xh, ge_t) & keep_t;
            const uint32_t re = (ge_bytes(d[k], xh, ge_hi) & keep_hi) | ~ge_bytes(d[k], xh, ge_lo);
            const int cnt = nvalid - 4 * k;
            const uint32_t keep = cnt >= 4 ? ~0u : (cnt <= 0 ? 0u : (1u << (8 * cnt)) - 1u);
            t[k] = (((rt >> 7) & 0x01010101u) * 0xffu) & keep;
            e[k] = (((re >> 7) & 0x01010101u) * 0xffu) & keep;
        }
        if (lane < 2 * cp.cnt) {
            const int64_t off = (int64_t)cp.w0 * 64 + lane * 32;
            uint4 *tb = (uint4 *)(a.bm[cp.img] + lv.bt_off + off);
            uint4 *eb = (uint4 *)(a.bm[cp.img] + lv.be_off + off);
            tb[0] = make_uint4(t[0], t[1], t[2], t[3]);
            tb[1] = make_uint4(t[4], t[5], t[6], t[7]);
            eb[0] = make_uint4(e[0], e[1], e[2], e[3]);
            eb[1] = make_uint4(e[4], e[5], e[6], e[7]);
        }
    }
}

// ---------------------------------------------------------------- search

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// One batch of kB reference rows of a work unit and, for each, the moving row
// one below it (ddy = -1): the lane's two reference words and kW words of the
// moving row around them (see search_unit_t).
template <int kB, int kW>
struct RowBatch {
    uint2 rt[kB], re[kB];
    uint32_t mt[kB][kW], me[kB][kW];
};

// The three horizontally shifted copies (ddx = -1, 0, +1 -> index 0, 1, 2) of
// one 32-pixel word k of a moving bitmap row: bits [t, t+32) of the row with
// t = 32k - (bx + ddx), from the row words m[0], m[1] (and m[2]) starting at
// word floor((32k - bx - 1) / 32); r = (32k - bx - 1) mod 32 (wave-uniform).
// kCase 0: r <= 29; kCase 1: r == 30; kCase 2: r == 31 (only this one needs m[2]).
template <int kCase>
__device__ __forceinline__ void shift3c(const uint32_t *m, uint32_t r, uint32_t *s)
{
    s[2] = funnel(m[1], m[0], r);
    if (kCase == 0) {
        s[1] = funnel(m[1], m[0], r + 1);
        s[0] = funnel(m[1], m[0], r + 2);
    } else if (kCase == 1) {
        s[1] = funnel(m[1], m[0], 31);
        s[0] = m[1];
    } else {
        s[1] = m[1];
        s[0] = funnel(m[2], m[1], 1);
    }
}

// Lanes of one row stream (CW = 2^cw_log2, each lane two words), units across
// a row and work units of a level, for `rows` rows per stream.
struct UnitPlan {
    int cw_log2, units_x, units;
};
__host__ __device__ __forceinline__ UnitPlan plan_level(const LevelGeom &lv, int rows, int cw_force)
{
    const int cols = lv.wpr;  // two-word columns per row (n32 / 2)
    // The stream width (8 .. 64 lanes) that pads the row least, ties going
    // wide; cw_force (3 .. 6, a launch-shape knob) overrides it.
    int best = 6, best_pad = 1 << 30;
    for (int c = 6; c >= 3; --c) {
        const int pad = (((cols + (1 << c) - 1) >> c) << c) - cols;
        if (pad < best_pad) {
            best = c;
            best_pad = pad;
        }
    }
    if (cw_force >= 3 && cw_force <= 6)
        best = cw_force;
    UnitPlan p;
    p.cw_log2 = best;
    p.units_x = (cols + (1 << best) - 1) >> best;
    const int rows_per_unit = rows * (kWave >> best);
    p.units = p.units_x * ((lv.h + rows_per_unit - 1) / rows_per_unit);
    return p;
}

// Nine candidate errors of one work unit.  A wavefront covers CW = 2^cw_log2
// lanes of two dword columns each and 64 / CW row streams; each stream walks
// `rows` rows (a multiple of kB, the same for every stream), kB at a time,
// with the next batch's loads in flight while one batch is scored.  Loads
// never branch: row and column indices are clamped into the level, and the
// exclusion words of anything outside it are masked to zero when the batch is
// scored (not when it is loaded, which would wait for the loads), zeroing
// those pixels' contribution whatever their threshold bits hold.
template <int kCase>
__device__ void search_unit_t(const uint8_t *ref, const uint8_t *mov, const LevelGeom &lv, int bx, int by,
                              int unit, int cw_log2, int rows, int units_x, uint32_t acc[9])
{
    constexpr int kB = kSearchBatch;        // rows per batch
    constexpr int kW = kCase == 2 ? 4 : 3;  // moving words per row for two reference words
    constexpr int kG = kW - 1;              // words the window may start before the row
    const int lane = threadIdx.x & 63;
    const int n32 = 2 * lv.wpr;
    const int h = lv.h;
    const int sx = unit % units_x, sy = unit / units_x;
    const int k = 2 * ((sx << cw_log2) + (lane & ((1 << cw_log2) - 1)));  // first of the lane's two words
    const int stream = lane >> cw_log2;
    const int y_begin = (sy * (kWave >> cw_log2) + stream) * rows;
    const int y_end = y_begin + rows < h ? y_begin + rows : h;  // y_end - 1 is a row of the level
    const uint8_t *tr = ref + lv.tb_off, *er = ref + lv.eb_off;
    const int u = -bx - 1;
    const int q = k + (u >> 5);  // arithmetic shift: floor((-bx - 1) / 32)
    const uint32_t r = (uint32_t)u & 31u;
    const int row_bytes = 4 * n32;

    // Per-lane column window and validity masks, fixed for the unit.  n32 is
    // even, so both reference words are in the row or neither is.  Where the
    // window q .. q+kW-1 lies wholly outside the row its start is clamped to
    // [-kG, n32 - 1] (every word stays masked); its words then lie within kG
    // words of the row, which the layout keeps inside the buffer (a 256-byte
    // guard precedes the first plane, the medians follow the last); tmg/emg
    // point kG words before the planes so offsets stay >= 0.
    const uint32_t kref = 4u * (uint32_t)(k < n32 ? k : n32 - 2);
    const uint32_t ref_ok = (k < n32 && y_begin < h) ? ~0u : 0u;
    const int qc = q < -kG ? -kG : (q > n32 - 1 ? n32 - 1 : q);
    const uint32_t coff = 4u * (uint32_t)(qc + kG);
    uint32_t cmask[kW];
#pragma unroll
    for (int i = 0; i < kW; ++i)
        cmask[i] = (q + i >= 0 && q + i < n32) ? ~0u : 0u;
    const uint8_t *tmg = mov + lv.tb_off - 4 * kG, *emg = mov + lv.eb_off - 4 * kG;
    auto load_moving = [&](int j, uint32_t *wt, uint32_t *we) {
        const int jc = j < 0 ? 0 : (j >= h ? h - 1 : j);
        const uint32_t off = (uint32_t)jc * (uint32_t)row_bytes + coff;
#pragma unroll
        for (int i = 0; i < kW; ++i) {
            wt[i] = *(const uint32_t *)(tmg + off + 4 * i);
            we[i] = *(const uint32_t *)(emg + off + 4 * i);
        }
    };
    // Exclusion words of moving row j with everything outside the level cleared.
    auto mask_moving = [&](int j, const uint32_t *we, uint32_t *out) {
        const uint32_t rmask = (uint32_t)j < (uint32_t)h ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < kW; ++i)
            out[i] = we[i] & cmask[i] & rmask;
    };
    auto load = [&](int y, RowBatch<kB, kW> &b) {
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            const int yy = y + i < y_end ? y + i : y_end - 1;
            const uint32_t base = (uint32_t)yy * (uint32_t)row_bytes + kref;
            b.rt[i] = *(const uint2 *)(tr + base);
            b.re[i] = *(const uint2 *)(er + base);
            // Past the stream's last row this re-reads that row's moving words
            // (cache hits); they are never scored.
            load_moving(yy - by + 1, b.mt[i], b.me[i]);
        }
    };

    // Shifted moving words seen by reference row y: rows y - by - ddy for
    // ddy = +1 (a*), 0 (b*); [word][ddx].
    uint32_t at[2][3], ae[2][3], bt[2][3], be[2][3];
    auto shift_row = [&](const uint32_t *mt, const uint32_t *me, uint32_t (*ct)[3], uint32_t (*ce)[3]) {
        shift3c<kCase>(mt, r, ct[0]);
        shift3c<kCase>(mt + 1, r, ct[1]);
        shift3c<kCase>(me, r, ce[0]);
        shift3c<kCase>(me + 1, r, ce[1]);
    };
    auto score = [&](const RowBatch<kB, kW> &b, int y) {
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            const uint32_t ok = y + i < y_end ? ref_ok : 0u;
            const uint32_t rt[2] = {b.rt[i].x, b.rt[i].y};
            const uint32_t re[2] = {b.re[i].x & ok, b.re[i].y & ok};
            uint32_t me[kW], ct[2][3], ce[2][3];
            mask_moving(y + i - by + 1, b.me[i], me);
            shift_row(b.mt[i], me, ct, ce);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    acc[d] += __builtin_popcount((rt[w] ^ ct[w][d]) & re[w] & ce[w][d]);      // ddy = -1
                    acc[3 + d] += __builtin_popcount((rt[w] ^ bt[w][d]) & re[w] & be[w][d]);  // ddy = 0
                    acc[6 + d] += __builtin_popcount((rt[w] ^ at[w][d]) & re[w] & ae[w][d]);  // ddy = +1
                }
            }
#pragma unroll
            for (int w = 0; w < 2; ++w)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    at[w][d] = bt[w][d];
                    ae[w][d] = be[w][d];
                    bt[w][d] = ct[w][d];
                    be[w][d] = ce[w][d];
                }
        }
    };

    // kP batches in a ring: while one is scored, the loads of the next kP - 1
    // are in flight.  Loads past the stream's rows are clamped to its last
    // row (valid addresses, cache hits) so that no load sits behind a branch;
    // the only branch, at the end of a round, is uniform (rows is).
    constexpr int kP = kSearchDepth;
    RowBatch<kB, kW> b[kP];
    {
        uint32_t w[4][kW], m[2][kW];
        load_moving(y_begin - by - 1, w[0], w[1]);
        load_moving(y_begin - by, w[2], w[3]);
#pragma unroll
        for (int k = 0; k < kP - 1; ++k)
            load(y_begin + k * kB, b[k]);
        mask_moving(y_begin - by - 1, w[1], m[0]);
        mask_moving(y_begin - by, w[3], m[1]);
        shift_row(w[0], m[0], at, ae);
        shift_row(w[2], m[1], bt, be);
    }
    for (int i = 0;; i += kP * kB) {
        const int y = y_begin + i;
#pragma unroll
        for (int k = 0; k < kP; ++k) {
            load(y + (k + kP - 1) * kB, b[(k + kP - 1) % kP]);
            score(b[k], y + k * kB);
        }
        if (i + kP * kB >= rows)
            break;
    }
}

__device__ __forceinline__ void search_unit(const uint8_t *ref, const uint8_t *mov, const LevelGeom &lv, int bx,
                                            int by, int unit, int cw_log2, int rows, int units_x, uint32_t acc[9])
{
    const uint32_t r = (uint32_t)(-bx - 1) & 31u;
    if (r <= 29)
        search_unit_t<0>(ref, mov, lv, bx, by, unit, cw_log2, rows, units_x, acc);
    else if (r == 30)
        search_unit_t<1>(ref, mov, lv, bx, by, unit, cw_log2, rows, units_x, acc);
    else
        search_unit_t<2>(ref, mov, lv, bx, by, unit, cw_log2, rows, units_x, acc);
}

// Sums each of v[0..N) over the wavefront (every lane gets the totals).
// Within each row of 16 lanes, DPP moves (no LDS): swap neighbours, swap
// pairs (quad permutes), mirror each half-row, mirror the row — after which
// every lane holds its row's sum; the last two steps cross rows with
// ds_bpermute, the N exchanges of a step all in flight at once.
template <int N>
__device__ __forceinline__ void wave_sums(uint32_t *v)
{
#pragma unroll
    for (int i = 0; i < N; ++i)  // quad_perm [1,0,3,2]
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0xb1, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // quad_perm [2,3,0,1]
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x4e, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // row_half_mirror
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x141, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // row_mirror
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x140, 0xf, 0xf, true);
#pragma unroll
    for (int d = 16; d <= 32; d <<= 1) {
        uint32_t o[N];
#pragma unroll
        for (int i = 0; i < N; ++i)
            o[i] = __shfl_xor(v[i], d);
#pragma unroll
        for (int i = 0; i < N; ++i)
            v[i] += o[i];
    }
}

// First minimum in ddy-major order; returns the candidate index 0..8.
__device__ __forceinline__ int argmin9(const uint32_t *c)
{
    int best = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (c[i] < c[best])
            best = i;
    return best;
}

__device__ __forceinline__ uint32_t *pair_state(const SearchArgs &a, int p)
{
    return a.state + (int64_t)p * a.state_stride;
}

__device__ __forceinline__ int32_t *pair_bases(const SearchArgs &a, int p)
{
    return (int32_t *)(pair_state(a, p) + (int64_t)a.g.L * kCounterWords);
}

__device__ __forceinline__ uint32_t *pair_surface(const SearchArgs &a, int p)
{
    return pair_state(a, p) + (int64_t)a.g.L * kCounterWords + 2 * a.g.L;
}

// Radius of the exhaustive window at the i-th coarsest level, and where its
// (2R+1)^2 surface starts.
__host__ __device__ __forceinline__ int coarse_radius(int i) { return (2 << i) - 1; }
__device__ __forceinline__ int coarse_surface_offset(int i)
{
    return i == 0 ? 0 : i == 1 ? 9 : i == 2 ? 58 : i == 3 ? 283 : 1244;
}

// Records level l's nine errors and chosen shift in pair p's output row.
__device__ __forceinline__ void write_level(const SearchArgs &a, int p, int l, const uint32_t *c, int sx, int sy)
{
    const SearchOutputs &o = a.out;
    const int64_t r = o.pair_image[p];
    const int L = a.g.L;
    if (o.trace)
        for (int i = 0; i < 9; ++i)
            o.trace[(r * L + l) * 9 + i] = c[i];
    if (o.level_shifts) {
        o.level_shifts[(r * L + l) * 2] = sx;
        o.level_shifts[(r * L + l) * 2 + 1] = sy;
    }
    if (l == 0) {
        o.shifts[2 * r] = sx;
        o.shifts[2 * r + 1] = sy;
        o.errs[r] = c[argmin9(c)];
    }
}

// Level 0's outputs for every pair, from its counters (the sum of their
// kCopies copies) and base.  Run by the last workgroup of the level-0 launch.
__device__ void finalize_level0(const SearchArgs &a)
{
    __shared__ uint32_t tot[kMaxStack * 9];
    for (int i = threadIdx.x; i < a.npairs * 9; i += blockDim.x) {
        const uint32_t *cnt = pair_state(a, i / 9) + i % 9;
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kCopies; ++k)
            s += load_shared(cnt + 9 * k);
        tot[i] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < a.npairs) {
        const int p = threadIdx.x;
        const uint32_t *c = tot + p * 9;
        const int32_t *bases = pair_bases(a, p);
        const int bx = (int32_t)load_shared((const uint32_t *)bases);
        const int by = (int32_t)load_shared((const uint32_t *)bases + 1);
        const int best = argmin9(c);
        write_level(a, p, 0, c, bx + best % 3 - 1, by + best / 3 - 1);
    }
}

// True in the workgroup that finishes last in the launch.  Tickets are taken
// in two stages so that no single counter receives more than about
// gridsize / kTicketGroups atomics: workgroup b counts into group b %
// kTicketGroups, and the last arrival of each group counts into t[G].
//
// Ordering without device-wide fences (which on gfx950 write back the whole
// L2): everything workgroups exchange within a launch is written and read
// with agent-scope atomics, performed at the coherence point.  Every thread
// first waits until its own memory operations have been acknowledged
// (vmcnt 0: stores and atomics performed), then the workgroup barrier, and
// only then does thread 0 take its ticket; each ticket counter is a single
// agent-scope atomic, so the workgroup that draws the last ticket observes
// every other workgroup's completed writes.  (A workgroup barrier alone does
// not wait for outstanding global writes.)
__device__ bool last_workgroup(uint32_t *t)
{
    __shared__ int s_last;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t n = gridDim.x * gridDim.y;
        const uint32_t b = blockIdx.y * gridDim.x + blockIdx.x;
        const uint32_t grp = b % kTicketGroups;
        const uint32_t members = (n - grp + kTicketGroups - 1) / kTicketGroups;
        const uint32_t groups = n < (uint32_t)kTicketGroups ? n : (uint32_t)kTicketGroups;
        s_last = 0;
        if (atomicAdd(t + grp, 1u) == members - 1)
            s_last = atomicAdd(t + kTicketGroups, 1u) == groups - 1;
    }
    __syncthreads();
    return s_last != 0;
}

// Column width (log2, in dwords) and row slabs of a coarse level handled by
// 256-lane workgroups: CW = 2^cw_log2 columns x 256 / CW row streams, each
// stream scoring 8 rows of a slab.
__host__ __device__ __forceinline__ int coarse_cw_log2(const LevelGeom &lv)
{
    int c = 0;
    while ((1 << c) < 2 * lv.wpr && c < 6)
        ++c;
    return c;
}

// Rows per stream of one coarse workgroup (all its loads are issued first).
// Four rather than eight: twice the workgroups, each with half the serial
// work, and more of them per compute unit to hide each other's latency.
constexpr int kCoarseRows = 4;

__host__ __device__ __forceinline__ int coarse_slab_rows(const LevelGeom &lv)
{
    return kCoarseRows * (256 >> coarse_cw_log2(lv));
}

__host__ __device__ __forceinline__ int coarse_slabs(const LevelGeom &lv)
{
    const int rows = coarse_slab_rows(lv);
    return (lv.h + rows - 1) / rows;
}

// Walks pair p's coarse error surfaces from the coarsest level down, testing
// the same nine candidates in the same order, with the same tie-break, as the
// nine-candidate search; records each level's outputs when `write` is set.
// The windows of radius 1, 3 and 7 are read from `surf` (their LDS copy), the
// larger ones from the pair's surfaces in memory.  Returns the shift chosen at
// the finest coarse level.
__device__ int2 coarse_walk(const SearchArgs &a, int p, const uint32_t *surf, bool write)
{
    int bx = 0, by = 0, sx = 0, sy = 0;
    for (int i = 0; i < a.coarse_n; ++i) {
        const int R = coarse_radius(i), side = 2 * R + 1;
        const bool lds = coarse_surface_offset(i) < kLdsSurfWords;
        const uint32_t *w = (lds ? surf : pair_surface(a, p)) + coarse_surface_offset(i);
        uint32_t c[9];
        // |bx|, |by| <= 2^(i+1) - 2 here, so every candidate lies in the window.
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const uint32_t *cell = w + (by + dy + R) * side + (bx + dx + R);
                c[(dy + 1) * 3 + dx + 1] = lds ? *cell : load_shared(cell);
            }
        const int best = argmin9(c);
        sx = bx + best % 3 - 1;
        sy = by + best / 3 - 1;
        if (write)
            write_level(a, p, a.g.L - 1 - i, c, sx, sy);
        bx = 2 * sx;
        by = 2 * sy;
    }
    return make_int2(sx, sy);
}

// Exhaustive search of the coarse levels.  The i-th coarsest level (i <
// coarse_n) is searched over every shift within radius R = 2^(i+1) - 1, which
// holds every candidate the coarse-to-fine search can test there.  Workgroup
// (item, pair) adds the errors of one row of a level's window (cy fixed,
// cx = -R..R) over one slab of rows into the pair's error surface.  The first
// fine level walks the surfaces; when every level is coarse, the last
// workgroup to finish walks them here and writes the outputs.
// The errors of one coarse item for every cx of its window row, added into
// the pair's error surface; kMaxR bounds the window radius R (7 or 31): words
// k-1 .. k+1 of a moving row hold every shift |cx| <= 31 of word k.
template <int kMaxR>
__device__ __forceinline__ void coarse_score(const SearchArgs &a, int pair, int i, int item)
{
    constexpr int kRows = kCoarseRows;
    __shared__ uint32_t red[4][2 * kMaxR + 1];
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    const LevelGeom &lv = g.lv[g.L - 1 - i];
    const int R = coarse_radius(i);
    const int slabs = coarse_slabs(lv);
    const int cy = item / slabs - R;
    const int y_lo = (item % slabs) * coarse_slab_rows(lv);
    const int n32 = 2 * lv.wpr, h = lv.h;
    const int row_bytes = 4 * n32;
    const uint8_t *tr = a.ref[pair] + lv.tb_off, *er = a.ref[pair] + lv.eb_off;
    // 4 bytes before the planes: column k-1 of row 0 stays inside the buffer
    // (the bitmap layout keeps a guard before the first plane).
    const uint8_t *tm4 = a.mov[pair] + lv.tb_off - 4, *em4 = a.mov[pair] + lv.eb_off - 4;

    const int cw_log2 = coarse_cw_log2(lv);
    const int cw = 1 << cw_log2;
    const int streams = 256 >> cw_log2;
    const int col = threadIdx.x & (cw - 1), stream = threadIdx.x >> cw_log2;

    uint32_t acc[2 * kMaxR + 1];
#pragma unroll
    for (int c = 0; c < 2 * kMaxR + 1; ++c)
        acc[c] = 0u;
    for (int k = col; k < n32; k += cw) {
        // Rows and columns outside the level are read clamped (or from the
        // neighbouring row) and their exclusion words masked below.
        const uint32_t cm0 = k >= 1 ? ~0u : 0u, cm2 = k + 1 < n32 ? ~0u : 0u;
        uint32_t t[kRows], e[kRows], mt[kRows][3], me[kRows][3];
#pragma unroll
        for (int b = 0; b < kRows; ++b) {
            const int y = y_lo + stream + b * streams;
            const int yc = y < h ? y : h - 1;
            const uint32_t ro = (uint32_t)yc * (uint32_t)row_bytes + 4u * (uint32_t)k;
            t[b] = *(const uint32_t *)(tr + ro);
            e[b] = *(const uint32_t *)(er + ro);
            const int j = y - cy;
            const int jc = j < 0 ? 0 : (j >= h ? h - 1 : j);
            const uint32_t mo = (uint32_t)jc * (uint32_t)row_bytes + 4u * (uint32_t)k;  // word k-1 at tm4 + mo
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                mt[b][w] = *(const uint32_t *)(tm4 + mo + 4 * w);
                me[b][w] = *(const uint32_t *)(em4 + mo + 4 * w);
            }
        }
#pragma unroll
        for (int b = 0; b < kRows; ++b) {
            const int y = y_lo + stream + b * streams;
            const uint32_t eb = y < h ? e[b] : 0u;
            const uint32_t rv = (uint32_t)(y - cy) < (uint32_t)h ? ~0u : 0u;
            const uint32_t m0 = me[b][0] & cm0 & rv, m1 = me[b][1] & rv, m2 = me[b][2] & cm2 & rv;
#pragma unroll
            for (int c = 0; c < 2 * kMaxR + 1; ++c) {
                const int cx = c - kMaxR;
                if (cx >= -R && cx <= R) {
                    const int o = 32 - cx;  // bit offset from the start of word k-1
                    const uint32_t st = o < 32 ? funnel(mt[b][1], mt[b][0], o) : funnel(mt[b][2], mt[b][1], o - 32);
                    const uint32_t se = o < 32 ? funnel(m1, m0, o) : funnel(m2, m1, o - 32);
                    acc[c] += __builtin_popcount((t[b] ^ st) & eb & se);
                }
            }
        }
    }
    wave_sums<2 * kMaxR + 1>(acc);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 2 * kMaxR + 1; ++c)
            red[wave][c] = acc[c];
    __syncthreads();
    uint32_t *surf = pair_surface(a, pair) + coarse_surface_offset(i);
    if ((int)threadIdx.x < 2 * R + 1) {
        const int c = threadIdx.x + kMaxR - R;
        const uint32_t v = red[0][c] + red[1][c] + red[2][c] + red[3][c];
        if (v)
            atomicAdd(surf + (cy + R) * (2 * R + 1) + threadIdx.x, v);
    }
}

// kMaxR: the largest window radius of the launch (7 for up to three coarse
// levels, 31 for five), which sizes the per-lane sums.
template <int kMaxR>
__global__ __launch_bounds__(256) void k_search_coarse(SearchArgs a)
{
    const int pair = blockIdx.y;
    const Geometry &g = a.g;
    int item = blockIdx.x, i = 0;
    for (;;) {
        const int cnt = (2 * coarse_radius(i) + 1) * coarse_slabs(g.lv[g.L - 1 - i]);
        if (item < cnt)
            break;
        item -= cnt;
        ++i;
    }
    if (kMaxR == 7 || coarse_radius(i) <= 7)
        coarse_score<7>(a, pair, i, item);
    else
        coarse_score<kMaxR>(a, pair, i, item);

    if (a.coarse_n < g.L || !last_workgroup(a.done))
        return;
    // Every level is coarse: walk all pairs' surfaces, the small windows
    // fetched into LDS at once.
    constexpr int kLoads = 8;
    __shared__ uint32_t ssurf[kMaxStack * kLdsSurfWords];
    const int words = a.npairs * kLdsSurfWords;
    for (int q0 = 0; q0 < words; q0 += 256 * kLoads) {
        uint32_t v[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            v[u] = q < words ? load_shared(pair_surface(a, q / kLdsSurfWords) + q % kLdsSurfWords) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            if (q < words)
                ssurf[q] = v[u];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < a.npairs)
        coarse_walk(a, threadIdx.x, ssurf + threadIdx.x * kLdsSurfWords, true);
}

// This level's base (twice the winner of the level above, or the coarse walk's
// result, or 0 at the top) into sbase[0..1] in LDS; one round trip.  Called by
// every thread of the workgroup; ends with a workgroup barrier.
__device__ __forceinline__ void level_base(const SearchArgs &a, int pair, int *sbase)
{
    __shared__ uint32_t cnt[kLdsSurfWords > kCounterWords ? kLdsSurfWords : kCounterWords];
    __shared__ uint32_t tot[9];
    __shared__ int sprev[2];
    const Geometry &g = a.g;
    const int l = a.level;
    uint32_t *state = pair_state(a, pair);
    int32_t *bases = pair_bases(a, pair);

    if (a.coarse_n > 0 && l == g.L - 1 - a.coarse_n) {
        // First level after the coarse ones: walk their surfaces.
        const uint32_t *surf = pair_surface(a, pair);
        uint32_t v[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = u * 256 + (int)threadIdx.x;
            v[u] = q < kLdsSurfWords ? surf[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = u * 256 + (int)threadIdx.x;
            if (q < kLdsSurfWords)
                cnt[q] = v[u];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int2 s = coarse_walk(a, pair, cnt, blockIdx.x == 0);
            sbase[0] = 2 * s.x;
            sbase[1] = 2 * s.y;
        }
    } else if (l < g.L - 1) {
        if (threadIdx.x < kCounterWords)
            cnt[threadIdx.x] = state[(l + 1) * kCounterWords + threadIdx.x];
        else if (threadIdx.x < kCounterWords + 2)
            sprev[threadIdx.x - kCounterWords] = bases[2 * (l + 1) + threadIdx.x - kCounterWords];
        __syncthreads();
        if (threadIdx.x < 9) {
            uint32_t s = 0;
#pragma unroll
            for (int k = 0; k < kCopies; ++k)
                s += cnt[k * 9 + threadIdx.x];
            tot[threadIdx.x] = s;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t c[9];
            for (int i = 0; i < 9; ++i)
                c[i] = tot[i];
            const int best = argmin9(c);
            const int sx = sprev[0] + best % 3 - 1, sy = sprev[1] + best / 3 - 1;
            sbase[0] = 2 * sx;
            sbase[1] = 2 * sy;
            if (blockIdx.x == 0)
                write_level(a, pair, l + 1, c, sx, sy);
        }
    } else if (threadIdx.x == 0) {
        sbase[0] = sbase[1] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x == 0 && l > 0) {
        // Read by the next level's launch.
        bases[2 * l] = sbase[0];
        bases[2 * l + 1] = sbase[1];
    } else if (threadIdx.x == 0 && blockIdx.x == 0) {
        // Read by this launch's last workgroup: published before its ticket.
        store_shared((uint32_t *)bases, (uint32_t)sbase[0]);
        store_shared((uint32_t *)bases + 1, (uint32_t)sbase[1]);
    }
}

// Sums the workgroup's nine errors into this level's counters (copy
// blockIdx.x % kCopies); at level 0 the last workgroup writes the outputs.
__device__ __forceinline__ void level_finish(const SearchArgs &a, int pair, const uint32_t *acc)
{
    __shared__ uint32_t red[4][9];
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    uint32_t v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        v[i] = acc[i];
    wave_sums<9>(v);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            red[wave][i] = v[i];
    __syncthreads();
    if (threadIdx.x < 9) {
        const uint32_t s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                           red[3][threadIdx.x];
        if (s)
            atomicAdd(pair_state(a, pair) + a.level * kCounterWords + (blockIdx.x % kCopies) * 9 + threadIdx.x, s);
    }
    if (a.level == 0 && last_workgroup(a.done + kTicketGroups + 1))
        finalize_level0(a);
}

// One level below the coarse ones, for every pair: grid (workgroups per pair, pairs).
__global__ __launch_bounds__(256) void k_search_fine(SearchArgs a)
{
    __shared__ int sbase[2];
    const int pair = blockIdx.y;
    level_base(a, pair, sbase);
    const LevelGeom &lv = a.g.lv[a.level];
    const UnitPlan p = plan_level(lv, a.rows_per_stream, a.cw_log2);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int unit = blockIdx.x * 4 + wave_id();
    if (unit < p.units)
        search_unit(a.ref[pair], a.mov[pair], lv, sbase[0], sbase[1], unit, p.cw_log2, a.rows_per_stream,
                    p.units_x, acc);
    level_finish(a, pair, acc);
}

// ---------------------------------------------------------------- one-workgroup search

// A pair whose bitmap pyramids fit LDS is searched by one workgroup of
// kSmallThreads lanes: both images' planes are copied into LDS once, then
// every level's nine candidates are scored there, the chosen shift feeding
// the next level without leaving the workgroup.
constexpr int kSmallThreads = 1024;

// The three words of moving row j around a column word's shifted window
// (words q .. q+2, q = k + floor((-bx - 1) / 32)) turned into the copies for
// ddx = -1, 0, +1 (shift3c; r = (-bx - 1) mod 32 fixes kCase).  Words outside
// the row, and rows outside the level, count with their exclusion bits
// cleared; their indices are clamped so that every read stays in the plane.
template <int kCase>
__device__ __forceinline__ void small_moving(const uint32_t *mT, const uint32_t *mE, int h, int n32, int j, int q,
                                             uint32_t r, uint32_t *st, uint32_t *se)
{
    const uint32_t rm = (uint32_t)j < (uint32_t)h ? ~0u : 0u;
    const int jc = j < 0 ? 0 : (j >= h ? h - 1 : j);
    uint32_t wt[3], we[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int w = q + i;
        const uint32_t cm = (w >= 0 && w < n32) ? rm : 0u;
        const int wc = w < 0 ? 0 : (w >= n32 ? n32 - 1 : w);
        wt[i] = mT[jc * n32 + wc];
        we[i] = mE[jc * n32 + wc] & cm;
    }
    shift3c<kCase>(wt, r, st);
    shift3c<kCase>(we, r, se);
}

// Adds the three ddx candidates of one ddy for a reference word pair (rt, re).
__device__ __forceinline__ void small_score3(uint32_t rt, uint32_t re, const uint32_t *st, const uint32_t *se,
                                             uint32_t *acc)
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        acc[d] += __builtin_popcount((rt ^ st[d]) & re & se[d]);
}

// Nine candidate errors of one level from LDS planes of h rows of n32 words
// (rT, rE: reference; mT, mE: moving) around the centre (bx, by), by the
// whole workgroup.  Work item (k, s) is column word k and the rows
// [s R, s R + R) of row stream s, walked top to bottom: reference row y meets
// moving rows y - by - ddy for ddy = +1, 0, -1, which are carried from one
// row to the next, so that each step loads one moving row.
template <int kCase>
__device__ void small_level(const uint32_t *rT, const uint32_t *rE, const uint32_t *mT, const uint32_t *mE,
                            int h, int n32, int bx, int by, uint32_t *acc)
{
    int S = n32 >= kSmallThreads ? 1 : kSmallThreads / n32;
    S = S < h ? S : h;
    const int R = (h + S - 1) / S;
    const int u = -bx - 1;
    const uint32_t r = (uint32_t)u & 31u;
    for (int item = threadIdx.x; item < n32 * S; item += kSmallThreads) {
        const int k = item % n32, s = item / n32;
        const int y0 = s * R, y1 = y0 + R < h ? y0 + R : h;
        const int q = k + (u >> 5);  // arithmetic shift: floor((-bx - 1) / 32)
        uint32_t at[3], ae[3], bt[3], be[3];
        small_moving<kCase>(mT, mE, h, n32, y0 - by - 1, q, r, at, ae);  // ddy = +1 for row y0
        small_moving<kCase>(mT, mE, h, n32, y0 - by, q, r, bt, be);      // ddy = 0
        for (int y = y0; y < y1; ++y) {
            uint32_t ct[3], ce[3];
            small_moving<kCase>(mT, mE, h, n32, y - by + 1, q, r, ct, ce);  // ddy = -1
            const uint32_t rt = rT[y * n32 + k], re = rE[y * n32 + k];
            small_score3(rt, re, ct, ce, acc);
            small_score3(rt, re, bt, be, acc + 3);
            small_score3(rt, re, at, ae, acc + 6);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                at[d] = bt[d];
                ae[d] = be[d];
                bt[d] = ct[d];
                be[d] = ce[d];
            }
        }
    }
}

// The same for a level of at most kSmallThreads (row, column word)
// positions: thread i takes position i (row-major), with its three moving
// rows loaded afresh.
template <int kCase>
__device__ void small_level_pos(const uint32_t *rT, const uint32_t *rE, const uint32_t *mT, const uint32_t *mE,
                                int h, int n32, int bx, int by, uint32_t *acc)
{
    const int pos = threadIdx.x;
    if (pos >= h * n32)
        return;
    const int u = -bx - 1;
    const uint32_t r = (uint32_t)u & 31u;
    const int y = pos / n32, k = pos - y * n32;
    const int q = k + (u >> 5);
    const uint32_t rt = rT[pos], re = rE[pos];
    uint32_t st[3], se[3], mt[3], me[3], nt[3], ne[3];
    small_moving<kCase>(mT, mE, h, n32, y - by + 1, q, r, st, se);  // ddy = -1
    small_moving<kCase>(mT, mE, h, n32, y - by, q, r, mt, me);      // ddy = 0
    small_moving<kCase>(mT, mE, h, n32, y - by - 1, q, r, nt, ne);  // ddy = +1
    small_score3(rt, re, st, se, acc);
    small_score3(rt, re, mt, me, acc + 3);
    small_score3(rt, re, nt, ne, acc + 6);
}

// Wave-uniform totals t[i] of v[i] over the wavefront: within each row of 16
// lanes DPP moves give every lane its row's sum (as in wave_sums), then the
// four rows' sums are read from lanes 0, 16, 32 and 48.
template <int N>
__device__ __forceinline__ void wave_totals(uint32_t *v, uint32_t *t)
{
#pragma unroll
    for (int i = 0; i < N; ++i)  // quad_perm [1,0,3,2]
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0xb1, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // quad_perm [2,3,0,1]
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x4e, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // row_half_mirror
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x141, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)  // row_mirror
        v[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[i], 0x140, 0xf, 0xf, true);
#pragma unroll
    for (int i = 0; i < N; ++i)
        t[i] = (uint32_t)__builtin_amdgcn_readlane((int)v[i], 0) + (uint32_t)__builtin_amdgcn_readlane((int)v[i], 16) +
               (uint32_t)__builtin_amdgcn_readlane((int)v[i], 32) + (uint32_t)__builtin_amdgcn_readlane((int)v[i], 48);
}

// Where one pair's results go (SearchOutputs resolved for its output row),
// read from the kernel arguments once at the start.
struct SmallOut {
    uint32_t *trace;      // null, or this row's L x 9 errors
    int32_t *lvs;         // null, or this row's L x 2 shifts
    int32_t *shift;       // this row's shift
    uint32_t *err;        // this row's error
};

// The level's shift from its nine (wave-uniform) totals, recorded by thread
// 0; (bx, by) moves to the next level's centre.
__device__ __forceinline__ void small_choose(const SmallOut &o, int l, const uint32_t *c, int &bx, int &by)
{
    const int best = argmin9(c);
    const int sx = bx + best % 3 - 1, sy = by + best / 3 - 1;
    if (threadIdx.x == 0) {
        if (o.trace)
            for (int i = 0; i < 9; ++i)
                o.trace[l * 9 + i] = c[i];
        if (o.lvs) {
            o.lvs[2 * l] = sx;
            o.lvs[2 * l + 1] = sy;
        }
        if (l == 0) {
            o.shift[0] = sx;
            o.shift[1] = sy;
            o.err[0] = c[best];
        }
    }
    bx = 2 * sx;
    by = 2 * sy;
}

// Level l by the whole workgroup.  Each wave adds its totals into tot[l % 3]
// with LDS atomics; after one barrier every lane reads the sums.  Thread 0
// clears the next level's buffer tot[(l - 1) % 3] before this barrier: its
// last readers (two levels up) read it before arriving at the previous
// level's barrier, which thread 0 has passed.
__device__ __forceinline__ void small_level_all(const SmallOut &o, int l, int4 lv, const uint32_t *ref,
                                                const uint32_t *mov, uint32_t (*tot)[9], int &bx, int &by)
{
    const int h = lv.x, n32 = lv.y, to = lv.z, eo = lv.w;
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t r = (uint32_t)(-bx - 1) & 31u;
    const uint32_t *rT = ref + to, *rE = ref + eo, *mT = mov + to, *mE = mov + eo;
    if (h * n32 <= kSmallThreads) {
        if (r <= 29)
            small_level_pos<0>(rT, rE, mT, mE, h, n32, bx, by, acc);
        else if (r == 30)
            small_level_pos<1>(rT, rE, mT, mE, h, n32, bx, by, acc);
        else
            small_level_pos<2>(rT, rE, mT, mE, h, n32, bx, by, acc);
    } else {
        if (r <= 29)
            small_level<0>(rT, rE, mT, mE, h, n32, bx, by, acc);
        else if (r == 30)
            small_level<1>(rT, rE, mT, mE, h, n32, bx, by, acc);
        else
            small_level<2>(rT, rE, mT, mE, h, n32, bx, by, acc);
    }
    uint32_t t[9];
    wave_totals<9>(acc, t);
    uint32_t *tb = tot[l % 3];
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (t[i])
                atomicAdd(&tb[i], t[i]);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            tot[(l + 2) % 3][i] = 0u;
    __syncthreads();
    uint32_t c[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        c[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)tb[i]);
    small_choose(o, l, c, bx, by);
}

// Grid: one workgroup per pair.  The bitmaps buffer of an image holds its
// planes between the leading guard and the medians, span = med_off - kAlign
// bytes; the reference's span goes to LDS offset 0, the moving image's after
// it, so that a plane's LDS offset is its buffer offset less kAlign.
constexpr int kSmallSpan16 = (int)(kSmallLdsBytes / 32);  // uint4 of one image's span, at most
constexpr int kStage = (kSmallSpan16 + kSmallThreads - 1) / kSmallThreads;

// A lane's share of one image's span, in named registers (loads of clang
// vector types stay in registers, where HIP's uint4 copies through memcpy and
// an array of them can land in scratch memory): elements f, f + kSmallThreads,
// ...; indices past the span are clamped to its last element, which is then
// stored several times over with the same value, so that no load sits behind
// a branch and every lane's loads are in flight together.
struct SmallStage {
    static_assert(kStage == 5, "five elements per lane");
    U32x4 v0, v1, v2, v3, v4;
    __device__ __forceinline__ static int at(int f, int j, int n16)
    {
        return f + j * kSmallThreads < n16 ? f + j * kSmallThreads : n16 - 1;
    }
    __device__ __forceinline__ void load(const U32x4 *src, int f, int n16)
    {
        v0 = src[at(f, 0, n16)];
        v1 = src[at(f, 1, n16)];
        v2 = src[at(f, 2, n16)];
        v3 = src[at(f, 3, n16)];
        v4 = src[at(f, 4, n16)];
    }
    __device__ __forceinline__ void store(U32x4 *dst, int f, int n16) const
    {
        dst[at(f, 0, n16)] = v0;
        dst[at(f, 1, n16)] = v1;
        dst[at(f, 2, n16)] = v2;
        dst[at(f, 3, n16)] = v3;
        dst[at(f, 4, n16)] = v4;
    }
};

__global__ __launch_bounds__(kSmallThreads) void k_search_small(SearchArgs a)
{
    __shared__ U32x4 planes[kSmallLdsBytes / 16];
    __shared__ uint32_t tot[3][9];
    __shared__ int4 s_lv[kMaxLevels];  // per level: rows, words per row, T and E plane offsets (words)
    __shared__ SmallOut s_out;
    const Geometry &g = a.g;
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    // Each level's geometry and the output addresses are read from the kernel
    // arguments once, while the planes load, and kept in LDS: the level loop
    // then makes no dependent argument load.
    const LevelGeom glv = g.lv[tid < g.L ? tid : 0];
    if (tid == 0) {
        const SearchOutputs &o = a.out;
        const int64_t r = o.pair_image[p];
        s_out.trace = o.trace ? o.trace + r * g.L * 9 : nullptr;
        s_out.lvs = o.level_shifts ? o.level_shifts + r * g.L * 2 : nullptr;
        s_out.shift = o.shifts + 2 * r;
        s_out.err = o.errs + r;
    }
    const int n16 = (int)((g.med_off - kAlign) / 16);
    SmallStage x, y;
    x.load((const U32x4 *)(a.ref[p] + kAlign), tid, n16);
    y.load((const U32x4 *)(a.mov[p] + kAlign), tid, n16);
    if (tid < g.L)
        s_lv[tid] = make_int4(glv.h, 2 * glv.wpr, (int)((glv.tb_off - kAlign) / 4), (int)((glv.eb_off - kAlign) / 4));
    if (tid < 27)
        (&tot[0][0])[tid] = 0u;
    x.store(planes, tid, n16);
    y.store(planes + n16, tid, n16);
    __syncthreads();
    const uint32_t *ref = (const uint32_t *)planes, *mov = ref + 4 * n16;
    const SmallOut o = s_out;
    int bx = 0, by = 0;
    for (int l = g.L - 1; l >= 0; --l)
        small_level_all(o, l, s_lv[l], ref, mov, tot, bx, by);
}

// Byte-map search (comparison path): each lane owns one dword (four pixels) of
// a reference row; a wavefront covers 64 dwords x `rows` rows.  The three
// horizontal shifts of a moving dword come from v_alignbyte over three
// consecutive dwords, the vertical ones from a window of three moving rows;
// each set byte of (T_r ^ S T_m) & E_r & S E_m holds 8 set bits, so the sums
// are divided by 8 at the end.  Loads are clamped and exclusion bytes masked
// as in the packed search.
__device__ void search_unit_bytes(const uint8_t *ref, const uint8_t *mov, const LevelGeom &lv, int bx, int by,
                                  int unit, int rows, int units_x, uint32_t acc[9])
{
    const int lane = threadIdx.x & 63;
    const int ncol = (int)(lv.gray_pitch / 4);  // dwords per row
    const int h = lv.h;
    const int sx = unit % units_x, sy = unit / units_x;
    const int k = sx * kWave + lane;
    const int y_begin = sy * rows;
    const int y_end = y_begin + rows < h ? y_begin + rows : h;
    const uint8_t *tr = ref + lv.bt_off, *er = ref + lv.be_off;
    const int64_t rb = lv.gray_pitch;
    const int u = -bx - 1;
    const int q = k + (u >> 2);  // floor((4k - bx - 1) / 4)
    const uint32_t r = (uint32_t)u & 3u;
    const uint32_t kref = 4u * (uint32_t)(k < ncol ? k : ncol - 1);
    const uint32_t ref_ok = (k < ncol && y_begin < h) ? ~0u : 0u;
    const int qc = q < -2 ? -2 : (q > ncol - 1 ? ncol - 1 : q);
    const uint32_t coff = 4u * (uint32_t)(qc + 2);
    uint32_t cmask[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        cmask[i] = (q + i >= 0 && q + i < ncol) ? ~0u : 0u;
    const uint8_t *tmg = mov + lv.bt_off - 8, *emg = mov + lv.be_off - 8;
    // Shifted moving dwords of row j for ddx = -1, 0, +1 (index 0, 1, 2).
    auto moving = [&](int j, uint32_t *st, uint32_t *se) {
        const int jc = j < 0 ? 0 : (j >= h ? h - 1 : j);
        const uint32_t rmask = j == jc ? ~0u : 0u;
        const uint32_t off = (uint32_t)jc * (uint32_t)rb + coff;
        uint32_t wt[3], we[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            wt[i] = *(const uint32_t *)(tmg + off + 4 * i);
            we[i] = *(const uint32_t *)(emg + off + 4 * i) & cmask[i] & rmask;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t o = r + 2u - (uint32_t)d;  // byte offset of shift ddx = d - 1 in the window
            const uint32_t lo = o >> 2, sh = o & 3u;
            st[d] = __builtin_amdgcn_alignbyte(lo ? wt[2] : wt[1], lo ? wt[1] : wt[0], sh);
            se[d] = __builtin_amdgcn_alignbyte(lo ? we[2] : we[1], lo ? we[1] : we[0], sh);
        }
    };
    uint32_t at[3], ae[3], bt[3], be[3];
    moving(y_begin - by + 1, at, ae);  // rotated below: a = ddy + 1 row, b = ddy 0 row
    moving(y_begin - by, bt, be);
    // Window: c* = row y - by + 1 (ddy = -1), b* = y - by (0), a* = y - by - 1 (+1).
    uint32_t ct[3], ce[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ct[d] = at[d];
        ce[d] = ae[d];
    }
    moving(y_begin - by - 1, at, ae);
    for (int y = y_begin; y < y_begin + rows; ++y) {
        const int yy = y < y_end ? y : y_end - 1;
        const uint32_t ok = y < y_end ? ref_ok : 0u;
        const uint32_t t0 = *(const uint32_t *)(tr + (uint32_t)yy * (uint32_t)rb + kref);
        const uint32_t e0 = *(const uint32_t *)(er + (uint32_t)yy * (uint32_t)rb + kref) & ok;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc[d] += __builtin_popcount((t0 ^ ct[d]) & e0 & ce[d]);      // ddy = -1
            acc[3 + d] += __builtin_popcount((t0 ^ bt[d]) & e0 & be[d]);  // ddy = 0
            acc[6 + d] += __builtin_popcount((t0 ^ at[d]) & e0 & ae[d]);  // ddy = +1
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            at[d] = bt[d];
            ae[d] = be[d];
            bt[d] = ct[d];
            be[d] = ce[d];
        }
        moving(y + 1 - by + 1, ct, ce);
    }
}

// One level of the byte-map search for every pair: grid (workgroups per pair, pairs).
__global__ __launch_bounds__(256) void k_search_bytes(SearchArgs a)
{
    __shared__ int sbase[2];
    const int pair = blockIdx.y;
    level_base(a, pair, sbase);
    const LevelGeom &lv = a.g.lv[a.level];
    const int ncol = (int)(lv.gray_pitch / 4);
    const int units_x = (ncol + kWave - 1) / kWave;
    const int units = units_x * ((lv.h + a.rows_per_stream - 1) / a.rows_per_stream);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int unit = blockIdx.x * 4 + wave_id();
    if (unit < units)
        search_unit_bytes(a.ref[pair], a.mov[pair], lv, sbase[0], sbase[1], unit, a.rows_per_stream, units_x,
                          acc);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        acc[i] >>= 3;  // eight set bits per counted pixel
    level_finish(a, pair, acc);
}

// ---------------------------------------------------------------- apply shifts

// One output byte o of a row: pixel o / 3, channel o % 3, from source row sy
// (already clamped when fill is 1; -1 when the whole row is outside for fill 0).
__device__ __forceinline__ uint8_t shifted_byte(const ApplyArgs &a, const uint8_t *src, int sy, int64_t o, int dx)
{
    const int64_t x = o / 3, c = o - 3 * x;
    int64_t sx = x - dx;
    if (sy < 0)
        return 0;
    if (sx < 0 || sx >= a.width) {
        if (a.fill == 0)
            return 0;
        sx = sx < 0 ? 0 : a.width - 1;
    }
    return src[(int64_t)sy * a.stride + 3 * sx + c];
}

// Workgroups walk the rows of all images (row r = image r / height, row
// r % height).  A thread writes 16 output bytes at a time: where those bytes
// come from 16 consecutive source bytes whose covering aligned dwords lie
// inside the source row, five aligned dword loads and v_alignbyte realign
// them; the rest (row ends, shifted-in pixels) goes byte by byte.
__global__ __launch_bounds__(256) void k_apply(ApplyArgs a)
{
    const int64_t rows = (int64_t)a.n * a.height;
    const int64_t row = 3 * (int64_t)a.width;
    for (int64_t rr = blockIdx.x; rr < rows; rr += gridDim.x) {
        const int img = (int)(rr / a.height);
        const int y = (int)(rr - (int64_t)img * a.height);
        const int dx = a.shifts[2 * img], dy = a.shifts[2 * img + 1];
        int sy = y - dy;
        if (sy < 0 || sy >= a.height)
            sy = a.fill == 1 ? (sy < 0 ? 0 : a.height - 1) : -1;
        const uint8_t *src = a.rgb[img];
        uint8_t *dst = a.out[img] + (int64_t)y * a.out_stride;
        const int64_t shift = 3 * (int64_t)dx;  // output byte o reads source byte o - shift
        const uint8_t *srow = sy >= 0 ? src + (int64_t)sy * a.stride : src;
        for (int64_t o = 16 * (int64_t)threadIdx.x; o < row; o += 16 * (int64_t)blockDim.x) {
            const int64_t s0 = o - shift;
            if (a.aligned && sy >= 0 && o + 16 <= row && s0 >= 0 && (s0 & ~3ll) + 20 <= row) {
                const uint32_t *w = (const uint32_t *)(srow + (s0 & ~3ll));
                const uint32_t r = (uint32_t)(s0 & 3);
                uint32_t v[5];
#pragma unroll
                for (int k = 0; k < 5; ++k)
                    v[k] = w[k];
                uint4 q;
                q.x = __builtin_amdgcn_alignbyte(v[1], v[0], r);
                q.y = __builtin_amdgcn_alignbyte(v[2], v[1], r);
                q.z = __builtin_amdgcn_alignbyte(v[3], v[2], r);
                q.w = __builtin_amdgcn_alignbyte(v[4], v[3], r);
                *(uint4 *)(dst + o) = q;
            } else {
                const int64_t end = o + 16 < row ? o + 16 : row;
                for (int64_t b = o; b < end; ++b)
                    dst[b] = shifted_byte(a, src, sy, b, dx);
            }
        }
    }
}

// ---------------------------------------------------------------- chained stacks

// Translations compose by addition: the shift of image i against the
// reference is its shift against its neighbour towards the reference plus
// that neighbour's shift against the reference.  One lane walks each side.
struct ChainArgs {
    int32_t *shifts;
    int32_t n, ref;
};

__global__ void k_chain(ChainArgs a)
{
    int32_t *shifts = a.shifts;
    const int n = a.n, ref = a.ref;
    if (threadIdx.x == 0) {
        for (int i = ref - 2; i >= 0; --i) {
            shifts[2 * i] += shifts[2 * (i + 1)];
            shifts[2 * i + 1] += shifts[2 * (i + 1) + 1];
        }
    } else if (threadIdx.x == 1) {
        for (int i = ref + 2; i < n; ++i) {
            shifts[2 * i] += shifts[2 * (i - 1)];
            shifts[2 * i + 1] += shifts[2 * (i - 1) + 1];
        }
    }
}

// ---------------------------------------------------------------- quadrant check

struct QuadFlagArgs {
    const int32_t *shifts;  // [4][2]
    int32_t *flag;
    int32_t tol, pad_;
};

__global__ void k_quadrant_flag(QuadFlagArgs a)
{
    if (threadIdx.x != 0)
        return;
    int32_t f = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            for (int c = 0; c < 2; ++c) {
                const int32_t d = a.shifts[2 * i + c] - a.shifts[2 * j + c];
                if (d > a.tol || -d > a.tol)
                    f = 1;
            }
    a.flag[0] = f;
}

}  // namespace

// ---------------------------------------------------------------- launchers

// Workgroups of 256 threads of kernel K that fit on one compute unit at once
// (registers and LDS), from the runtime's occupancy calculator; cached once
// per kernel (each instantiation has its own cache, so kernels that share an
// argument type do not share a value).
template <auto K, int kThreads = 256>
int resident_per_cu()
{
    static std::atomic<int> cached{0};
    int v = cached.load(std::memory_order_relaxed);
    if (v == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, K, kThreads, 0) != hipSuccess || n < 1)
            n = 1;
        cached.store(n, std::memory_order_relaxed);
        v = n;
    }
    return v;
}

hipError_t launch_zero(const ZeroArgs &a, hipStream_t s)
{
    if (a.count <= 0)
        return hipSuccess;
    int64_t most = 0;
    for (int i = 0; i < a.count; ++i)
        most = a.words[i] > most ? a.words[i] : most;
    int blocks = (int)((most + 255) / 256);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    return launch_kernel("k_zero", k_zero, dim3(blocks, a.count), dim3(256), s, a);
}

hipError_t launch_pyramid(const PyramidArgs &in, int cus, hipStream_t s, int slots_pct, int group_log2)
{
    PyramidArgs a = in;
    a.tiles_x = (a.g.W + kTileW - 1) / kTileW;
    a.tiles_y = (a.g.H + kTileH - 1) / kTileH;
    a.group_log2 = group_log2;
    const int64_t total = (int64_t)a.tiles_x * a.tiles_y * a.n;
    // One round of resident workgroups (scaled by slots_pct); each XCD gets
    // the same number of slots (see k_pyramid), at most one per tile group.
    const int64_t share = (total + kXcds - 1) / kXcds;
    const int64_t groups = (share + (1 << group_log2) - 1) >> group_log2;
    int64_t slots = (int64_t)cus * resident_per_cu<k_pyramid>() * slots_pct / (100 * kXcds);
    slots = slots > groups ? groups : (slots < 1 ? 1 : slots);
    a.xcd_tiles = (int32_t)share;
    const int blocks = (int)(slots * kXcds);
    a.merge = blocks >= kMergeMinWgsPerImage * a.n;
    note_pyramid_launch(blocks, a.merge);
    hipError_t e = launch_kernel("k_pyramid", k_pyramid, dim3(blocks), dim3(256), s, a);
    if (e != hipSuccess || a.g.L <= kFused)
        return e;
    CoarsePyramidArgs c;
    for (int i = 0; i < a.n; ++i)
        c.pyr[i] = a.pyr[i];
    c.n = a.n;
    c.pad_ = 0;
    c.g = a.g;
    return launch_kernel("k_pyramid_coarse", k_pyramid_coarse, dim3(a.n), dim3(256), s, c);
}

hipError_t launch_chain(int32_t *d_shifts, int n, int ref, hipStream_t s)
{
    return launch_kernel("k_chain", k_chain, dim3(1), dim3(64), s, ChainArgs{d_shifts, n, ref});
}

hipError_t launch_quadrant_flag(const int32_t *d_shifts, int32_t tol, int32_t *d_flag, hipStream_t s)
{
    return launch_kernel("k_quadrant_flag", k_quadrant_flag, dim3(1), dim3(64), s,
                         QuadFlagArgs{d_shifts, d_flag, tol, 0});
}

hipError_t launch_apply(const ApplyArgs &a, int cus, hipStream_t s)
{
    const int64_t rows = (int64_t)a.n * a.height;
    const int64_t cap = (int64_t)cus * 64;
    const int64_t blocks = rows < cap ? rows : cap;
    return launch_kernel("k_apply", k_apply, dim3((unsigned)blocks), dim3(256), s, a);
}

hipError_t launch_bytemaps(const BitmapArgs &a, int cus, hipStream_t s)
{
    const int64_t total = a.chunk_start[a.g.L] * a.n;
    int64_t blocks = (total + 3) / 4;
    const int64_t cap = (int64_t)cus * resident_per_cu<k_bytemaps>();
    blocks = blocks > cap ? cap : (blocks < 1 ? 1 : blocks);
    return launch_kernel("k_bytemaps", k_bytemaps, dim3((unsigned)blocks), dim3(256), s, a);
}

hipError_t launch_search_bytes(SearchArgs a, int cus, hipStream_t s)
{
    const Geometry &g = a.g;
    a.coarse_n = 0;
    const int64_t resident = (int64_t)cus * resident_per_cu<k_search_bytes>();
    for (int l = g.L - 1; l >= 0; --l) {
        const LevelGeom &lv = g.lv[l];
        const int units_x = (int)((lv.gray_pitch / 4 + kWave - 1) / kWave);
        auto blocks_for = [&](int rows) {
            const int units = units_x * ((lv.h + rows - 1) / rows);
            return ((units + 3) / 4 + kXcds - 1) / kXcds * kXcds;
        };
        int rows = 4;
        while (rows < 256 && (int64_t)blocks_for(rows) * a.npairs > resident)
            rows += 4;
        a.level = l;
        a.rows_per_stream = rows;
        const hipError_t e = launch_kernel("k_search_bytes", k_search_bytes, dim3(blocks_for(rows), a.npairs),
                                           dim3(256), s, a);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int kW, bool kPairs>
hipError_t launch_bitmaps_w(const BitmapArgs &a, int cus, hipStream_t s, int blocks_pct)
{
    const int64_t total = a.chunk_start[a.g.L] * a.n;
    int64_t blocks = (total + kW - 1) / kW;
    const int64_t cap = (int64_t)cus * resident_per_cu<k_bitmaps<kW, kPairs>, 64 * kW>() * blocks_pct / 100;
    blocks = blocks > cap ? cap : (blocks < 1 ? 1 : blocks);
    return launch_kernel("k_bitmaps", k_bitmaps<kW, kPairs>, dim3((unsigned)blocks), dim3(64 * kW), s, a);
}

template <bool kPairs>
hipError_t launch_bitmaps_p(const BitmapArgs &a, int cus, hipStream_t s, int blocks_pct, int waves)
{
    // Wavefronts walk their items independently; the workgroup size only
    // changes how the launch is cut (a launch-shape knob).
    if (waves == 2)
        return launch_bitmaps_w<2, kPairs>(a, cus, s, blocks_pct);
    if (waves == 8)
        return launch_bitmaps_w<8, kPairs>(a, cus, s, blocks_pct);
    return launch_bitmaps_w<4, kPairs>(a, cus, s, blocks_pct);
}

hipError_t launch_bitmaps(const BitmapArgs &a, int cus, hipStream_t s, int blocks_pct, int waves)
{
    return a.pairs ? launch_bitmaps_p<true>(a, cus, s, blocks_pct, waves)
                   : launch_bitmaps_p<false>(a, cus, s, blocks_pct, waves);
}

// The built-in rule searches the i-th coarsest level exhaustively when i < 3
// and its window rows stay cheap for one workgroup: at most kCoarseDwords
// dwords.  The windows of radius 15 and 31 (i = 3, 4) are taken only when a
// launch shape asks for them: on a mix of small stacks they cost more than
// the fine launches they replace, and pairs small enough to gain from them
// are searched by one workgroup instead.
constexpr int64_t kCoarseDwords = 8192;
constexpr int kCoarseRule = 3;

int coarse_level_count(const Geometry &g, int npairs)
{
    (void)npairs;
    int cn = 0;
    while (cn < kCoarseRule && cn < g.L && (int64_t)2 * g.lv[g.L - 1 - cn].wpr * g.lv[g.L - 1 - cn].h <= kCoarseDwords)
        ++cn;
    return cn;
}

// Workgroups per pair of one fine level.  Workgroups are dealt to the XCDs
// in turn, so with a row of blocks whose length is a multiple of kXcds every
// pair's workgroup for one unit runs on the same XCD, whose L2 then serves
// the shared reference rows.
int search_row_blocks(const Geometry &g, int l, int rows, int cw_log2)
{
    return ((plan_level(g.lv[l], rows, cw_log2).units + 3) / 4 + kXcds - 1) / kXcds * kXcds;
}

int search_rows_rule(const Geometry &g, int l, int npairs, int cus, int cw_log2)
{
    // Rows per stream: the fewest (a multiple of the batches in flight) that
    // keep the grid within one round of resident workgroups, so that every
    // compute unit holds about as many workgroups as it can run and none
    // waits for another to finish.
    static_assert(kRowsStep == kSearchBatch * kSearchDepth, "rows per stream fill whole batches");
    const int64_t resident = (int64_t)cus * resident_per_cu<k_search_fine>();
    int rows = kRowsStep;
    while (rows < kRowsMax && (int64_t)search_row_blocks(g, l, rows, cw_log2) * npairs > resident)
        rows += kRowsStep;
    return rows;
}

int coarse_levels_used(const Geometry &g, int npairs, const LaunchTune *t)
{
    if (!t || t->coarse < 0)
        return coarse_level_count(g, npairs);
    const int most = g.L < kCoarseLevels ? g.L : kCoarseLevels;
    return t->coarse < most ? t->coarse : most;
}

bool small_search_fits(const Geometry &g) { return 2 * (g.med_off - kAlign) <= kSmallLdsBytes; }

bool small_search_used(const Geometry &g, const LaunchTune *t)
{
    return (!t || t->small != 0) && small_search_fits(g);
}

hipError_t launch_search(SearchArgs a, int cus, hipStream_t s, const LaunchTune *t)
{
    const Geometry &g = a.g;
    if (small_search_used(g, t))
        return launch_kernel("k_search_small", k_search_small, dim3(a.npairs), dim3(kSmallThreads), s, a);
    const int cn = coarse_levels_used(g, a.npairs, t);
    a.coarse_n = cn;
    hipError_t e = hipSuccess;
    if (cn > 0) {
        int items = 0;
        for (int i = 0; i < cn; ++i)
            items += (2 * coarse_radius(i) + 1) * coarse_slabs(g.lv[g.L - 1 - i]);
        e = launch_kernel("k_search_coarse", cn > 3 ? k_search_coarse<31> : k_search_coarse<7>, dim3(items, a.npairs),
                          dim3(256), s, a);
        if (e != hipSuccess)
            return e;
    }
    for (int l = g.L - 1 - cn; l >= 0; --l) {
        const int cw = t ? t->cw[l] : 0;
        const int rows = t && t->rows[l] > 0 ? t->rows[l] : search_rows_rule(g, l, a.npairs, cus, cw);
        a.level = l;
        a.rows_per_stream = rows;
        a.cw_log2 = cw;
        e = launch_kernel("k_search_fine", k_search_fine, dim3(search_row_blocks(g, l, rows, cw), a.npairs),
                          dim3(256), s, a);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace mtb
