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

#include "mtb_internal.h"

namespace mtb {

namespace {

constexpr int kWave = 64;

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

// Workgroup tile: kTileH = 64 rows x kTileW = 256 columns of level 0.  Wave w
// owns rows 16w .. 16w+15; lane (bx = lane & 15, by = lane >> 4) owns the
// 4-row x 16-column block at (X0 + 16 bx, Y0 + 16 w + 4 by).  Levels 1 and 2
// stay inside the lane, levels 3 and 4 combine lanes of the wave with
// shuffles, levels 5 and 6 combine the four waves through LDS.  Each lane
// reads 4 x 48 bytes of RGB per tile; a row of 16 lanes covers 768
// contiguous bytes.
__global__ __launch_bounds__(256) void k_pyramid(PyramidArgs a)
{
    __shared__ uint32_t hist01[4][2][256];        // per wave, levels 0 and 1
    __shared__ uint32_t histc[kFused - 2][256];   // levels 2 .. 6, whole workgroup
    __shared__ uint32_t lvl4[2][4][16];           // level-4 pixels of a tile, by tile parity

    const int tid = threadIdx.x;
    const int wave = wave_id();
    const int lane = tid & 63;
    const int bx = lane & 15, by = lane >> 4;
    const Geometry &g = a.g;
    const int fused = g.L < kFused ? g.L : kFused;

    for (int i = tid; i < 4 * 2 * 256; i += 256)
        (&hist01[0][0][0])[i] = 0u;
    for (int i = tid; i < (kFused - 2) * 256; i += 256)
        (&histc[0][0])[i] = 0u;
    __syncthreads();

    const int64_t per_image = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t total = per_image * a.n;
    const int64_t t0 = (int64_t)blockIdx.x * a.tiles_per_block;
    const int64_t t1 = t0 + a.tiles_per_block < total ? t0 + a.tiles_per_block : total;

    auto flush = [&](int img) {
        __syncthreads();
        uint32_t *gh = (uint32_t *)(a.pyr[img] + g.hist_off);
        for (int l = 0; l < fused; ++l) {
            uint32_t s;
            if (l < 2) {
                s = hist01[0][l][tid] + hist01[1][l][tid] + hist01[2][l][tid] + hist01[3][l][tid];
                hist01[0][l][tid] = hist01[1][l][tid] = hist01[2][l][tid] = hist01[3][l][tid] = 0u;
            } else {
                s = histc[l - 2][tid];
                histc[l - 2][tid] = 0u;
            }
            if (s)
                atomicAdd(gh + l * 256 + tid, s);
        }
        __syncthreads();
    };

    int cur = -1;
    int parity = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const int img = (int)(t / per_image);
        if (img != cur) {
            if (cur >= 0)
                flush(cur);
            cur = img;
        }
        const int64_t r = t - (int64_t)img * per_image;
        const int tx = (int)(r % a.tiles_x), ty = (int)(r / a.tiles_x);
        const int X0 = tx * kTileW, Y0 = ty * kTileH;
        const int x0 = X0 + 16 * bx, y0 = Y0 + 16 * wave + 4 * by;
        const uint8_t *rgb = a.rgb[img];
        uint8_t *pyr = a.pyr[img];
        const bool full = x0 + 15 < g.W;

        // ---- level 0: gray of the 4x16 block; all loads issued before any use
        uint32_t gv[4][16];
        if (a.align == 16 && full) {
            uint4 q[4][3];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                if (y0 + rr < g.H) {
                    const uint4 *p = (const uint4 *)(rgb + (int64_t)(y0 + rr) * a.stride + 3 * (int64_t)x0);
                    q[rr][0] = p[0];
                    q[rr][1] = p[1];
                    q[rr][2] = p[2];
                } else {
                    q[rr][0] = q[rr][1] = q[rr][2] = make_uint4(0u, 0u, 0u, 0u);
                }
            }
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
        {
            const LevelGeom &lv = g.lv[0];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int y = y0 + rr;
                if (y < g.H && x0 < g.W) {
                    // x0 % 16 == 0, x0 < W <= pitch, pitch % 64 == 0: 16 bytes inside the row.
                    *(uint4 *)(pyr + lv.gray_off + (int64_t)y * lv.gray_pitch + x0) =
                        make_uint4(pack4(&gv[rr][0]), pack4(&gv[rr][4]), pack4(&gv[rr][8]), pack4(&gv[rr][12]));
                    if (full) {
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            atomicAdd(&hist01[wave][0][gv[rr][c]], 1u);
                    } else {
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            if (x0 + c < g.W)
                                atomicAdd(&hist01[wave][0][gv[rr][c]], 1u);
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
                    *(uint2 *)(pyr + l1.gray_off + (int64_t)(y1 + i) * l1.gray_pitch + x1) =
                        make_uint2(pack4(&u1[i][0]), pack4(&u1[i][4]));
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (x1 + j < l1.w)
                            atomicAdd(&hist01[wave][1][u1[i][j]], 1u);
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
                            // ---- levels 5 and 6: the tile holds 4 x 16 level-4 pixels
                            // (row = wave, column = bx).
                            if (by == 0)
                                lvl4[parity][wave][bx] = u4;
                            __syncthreads();
                            const uint32_t(*q)[16] = lvl4[parity];
                            if (tid < 16) {
                                const int i5 = tid >> 3, j5 = tid & 7;
                                const uint32_t u5 = (q[2 * i5][2 * j5] + q[2 * i5][2 * j5 + 1] +
                                                     q[2 * i5 + 1][2 * j5] + q[2 * i5 + 1][2 * j5 + 1]) >> 2;
                                const LevelGeom &l5 = g.lv[5];
                                const int x5 = (X0 >> 5) + j5, y5 = (Y0 >> 5) + i5;
                                if (y5 < l5.h && x5 < l5.w) {
                                    pyr[l5.gray_off + (int64_t)y5 * l5.gray_pitch + x5] = (uint8_t)u5;
                                    atomicAdd(&histc[3][u5], 1u);
                                }
                            } else if (fused > 6 && tid >= 64 && tid < 68) {
                                const int j6 = tid - 64;
                                uint32_t s6 = 0;
#pragma unroll
                                for (int i = 0; i < 2; ++i)
#pragma unroll
                                    for (int j = 2 * j6; j < 2 * j6 + 2; ++j)
                                        s6 += (q[2 * i][2 * j] + q[2 * i][2 * j + 1] + q[2 * i + 1][2 * j] +
                                               q[2 * i + 1][2 * j + 1]) >> 2;
                                const uint32_t u6 = s6 >> 2;
                                const LevelGeom &l6 = g.lv[6];
                                const int x6 = (X0 >> 6) + j6, y6 = Y0 >> 6;
                                if (y6 < l6.h && x6 < l6.w) {
                                    pyr[l6.gray_off + (int64_t)y6 * l6.gray_pitch + x6] = (uint8_t)u6;
                                    atomicAdd(&histc[4][u6], 1u);
                                }
                            }
                            parity ^= 1;
                        }
                    }
                }
            }
        }
    }
    if (cur >= 0)
        flush(cur);
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

// Lower median of a 256-bin histogram holding npix pixels, computed by one
// wavefront: smallest v whose cumulative count reaches ceil(npix / 2).
__device__ uint32_t wave_median(const uint32_t *hist, uint32_t npix)
{
    const int lane = threadIdx.x & 63;
    const uint4 h = *(const uint4 *)(hist + 4 * lane);
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
    return __shfl(v, f < 0 ? 0 : f);
}

// Moves a wave-uniform 32-bit value into one lane of a vector register.
#define MTB_WRITELANE(dst, val, lane_imm) \
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(dst) : "s"(val), "i"(lane_imm))

struct ChunkPos {
    int img, level, w0, cnt;
};

__device__ __forceinline__ ChunkPos chunk_pos(const BitmapArgs &a, int64_t c, int64_t per_image)
{
    ChunkPos p;
    p.img = (int)(c / per_image);
    const int64_t cc = c - (int64_t)p.img * per_image;
    int l = 0;
    while (cc >= a.chunk_start[l + 1])
        ++l;
    p.level = l;
    p.w0 = (int)(cc - a.chunk_start[l]) * kChunkWords;
    const int nwords = a.g.lv[l].h * a.g.lv[l].wpr;
    p.cnt = nwords - p.w0 < kChunkWords ? nwords - p.w0 : kChunkWords;
    return p;
}

__device__ __forceinline__ void load_chunk(const BitmapArgs &a, const ChunkPos &p, int lane, uint4 &v0, uint4 &v1)
{
    const uint8_t *src = a.pyr[p.img] + a.g.lv[p.level].gray_off + (int64_t)p.w0 * 64 + lane * 32;
    const int bytes = p.cnt * 64;
    v0 = lane * 32 < bytes ? ((const uint4 *)src)[0] : make_uint4(0u, 0u, 0u, 0u);
    v1 = lane * 32 + 16 < bytes ? ((const uint4 *)src)[1] : make_uint4(0u, 0u, 0u, 0u);
}

// Each wavefront walks a contiguous run of chunks of kChunkWords = 32
// consecutive 64-pixel words of one level.  Lane i loads bytes [32 i, 32 i +
// 32) of the chunk (the next chunk's load is issued before the current one is
// processed); the chunk is staged in LDS and read back byte-transposed
// (lane i <- byte 64 j + i), so that one ballot yields word j.  T words land
// in lanes 0..31 and E words in lanes 32..63, and one store writes both.
__global__ __launch_bounds__(256) void k_bitmaps(BitmapArgs a)
{
    __shared__ uint4 stage[4][2 * kWave];
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
    const uint8_t *st = (const uint8_t *)&stage[wave][0];

    int cur_img = -1, cur_l = -1;
    uint32_t m = 0;
    ChunkPos p = chunk_pos(a, c0, per_image);
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
        }
        if (cp.w0 == 0 && lane == 0)
            ((int32_t *)(a.bm[cp.img] + g.med_off))[cp.level] = (int32_t)m;

        __builtin_amdgcn_wave_barrier();
        stage[wave][2 * lane] = v0;
        stage[wave][2 * lane + 1] = v1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        if (c + 1 < c1) {
            p = chunk_pos(a, c + 1, per_image);
            load_chunk(a, p, lane, v0, v1);
        }

        // Bits past the level width are zero: only the last word of a row is partial.
        const int tail = lv.w & 63;
        const uint64_t last_mask = tail ? ((1ull << tail) - 1ull) : ~0ull;
        int k = cp.w0 % lv.wpr;
        uint32_t out_lo = 0, out_hi = 0;
        const uint32_t ebias = X - m;
        uint32_t gvs[kChunkWords];  // all reads issued before the first use
#pragma unroll
        for (int j = 0; j < kChunkWords; ++j)
            gvs[j] = st[j * 64 + lane];
#pragma unroll
        for (int j = 0; j < kChunkWords; ++j) {
            if (j < cp.cnt) {
                const uint32_t gv = gvs[j];
                const uint64_t vm = k == lv.wpr - 1 ? last_mask : ~0ull;
                const uint64_t tw = ballot(gv > m) & vm;
                const uint64_t ew = ballot(gv + ebias > 2u * X) & vm;
                const uint32_t tlo = (uint32_t)tw, thi = (uint32_t)(tw >> 32);
                const uint32_t elo = (uint32_t)ew, ehi = (uint32_t)(ew >> 32);
                MTB_WRITELANE(out_lo, tlo, j);
                MTB_WRITELANE(out_hi, thi, j);
                MTB_WRITELANE(out_lo, elo, j + 32);
                MTB_WRITELANE(out_hi, ehi, j + 32);
                if (++k == lv.wpr)
                    k = 0;
            }
        }
        const uint64_t word = ((uint64_t)out_hi << 32) | out_lo;
        if (lane < 32) {
            if (lane < cp.cnt)
                ((uint64_t *)(a.bm[cp.img] + lv.tb_off))[cp.w0 + lane] = word;
        } else if (lane - 32 < cp.cnt) {
            ((uint64_t *)(a.bm[cp.img] + lv.eb_off))[cp.w0 + lane - 32] = word;
        }
    }
}

// ---------------------------------------------------------------- search

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// The three horizontally shifted copies (ddx = -1, 0, +1 -> index 0, 1, 2) of
// one 32-pixel word of a moving bitmap row: bits [t, t+32) of the row with
// t = 32k - (bx + ddx), from the three row words m0, m1, m2 starting at word
// floor((32k - bx - 1) / 32); r = (32k - bx - 1) mod 32.
__device__ __forceinline__ void shift3(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t r, uint32_t *s)
{
    s[2] = funnel(m1, m0, r);
    s[1] = r + 1 < 32 ? funnel(m1, m0, r + 1) : m1;
    s[0] = r + 2 < 32 ? funnel(m1, m0, r + 2) : funnel(m2, m1, r + 2 - 32);
}

// Loads the three row words for shift3 (zero outside the row and outside the level).
__device__ __forceinline__ void load3(const uint32_t *plane, int j, int h, int n32, int q, uint32_t *w)
{
    w[0] = w[1] = w[2] = 0u;
    if (j >= 0 && j < h) {
        const uint32_t *p = plane + j * n32;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (q + i >= 0 && q + i < n32)
                w[i] = p[q + i];
    }
}

// Nine candidate errors of one work unit.  A wavefront covers CW = 2^cw_log2
// dword columns and 64 / CW row streams; each stream walks `rows` rows.  Rows
// are processed four at a time with all of their loads issued first.
__device__ void search_unit(const uint8_t *ref, const uint8_t *mov, const LevelGeom &lv, int bx,
                            int by, int unit, int cw_log2, int rows, int units_x, uint32_t acc[9])
{
    const int lane = threadIdx.x & 63;
    const int n32 = 2 * lv.wpr;
    const int h = lv.h;
    const int sx = unit % units_x, sy = unit / units_x;
    const int k = (sx << cw_log2) + (lane & ((1 << cw_log2) - 1));
    const int stream = lane >> cw_log2;
    const int y_begin = (sy * (kWave >> cw_log2) + stream) * rows;
    const int y_end = y_begin + rows < h ? y_begin + rows : h;
    if (y_begin >= h)
        return;
    const uint32_t *tr = (const uint32_t *)(ref + lv.tb_off);
    const uint32_t *er = (const uint32_t *)(ref + lv.eb_off);
    const uint32_t *tm = (const uint32_t *)(mov + lv.tb_off);
    const uint32_t *em = (const uint32_t *)(mov + lv.eb_off);
    const int u = -bx - 1;
    const int q = k + (u >> 5);           // arithmetic shift: floor((-bx - 1) / 32)
    const uint32_t r = (uint32_t)u & 31u;
    const bool col_ok = k < n32;

    // Moving rows seen by reference row y: y - by - ddy for ddy = +1, 0, -1.
    uint32_t at[3], ae[3], bt[3], be[3];
    {
        uint32_t w[3];
        load3(tm, y_begin - by - 1, h, n32, q, w);
        shift3(w[0], w[1], w[2], r, at);
        load3(em, y_begin - by - 1, h, n32, q, w);
        shift3(w[0], w[1], w[2], r, ae);
        load3(tm, y_begin - by, h, n32, q, w);
        shift3(w[0], w[1], w[2], r, bt);
        load3(em, y_begin - by, h, n32, q, w);
        shift3(w[0], w[1], w[2], r, be);
    }
    for (int y = y_begin; y < y_end; y += 4) {
        uint32_t rt[4], re[4], mt[4][3], me[4][3];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool ok = y + i < y_end;
            rt[i] = (ok && col_ok) ? tr[(y + i) * n32 + k] : 0u;
            re[i] = (ok && col_ok) ? er[(y + i) * n32 + k] : 0u;
            load3(tm, ok ? y + i - by + 1 : -1, h, n32, q, mt[i]);
            load3(em, ok ? y + i - by + 1 : -1, h, n32, q, me[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t ct[3], ce[3];
            shift3(mt[i][0], mt[i][1], mt[i][2], r, ct);
            shift3(me[i][0], me[i][1], me[i][2], r, ce);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                acc[d] += __builtin_popcount((rt[i] ^ ct[d]) & re[i] & ce[d]);      // ddy = -1
                acc[3 + d] += __builtin_popcount((rt[i] ^ bt[d]) & re[i] & be[d]);  // ddy = 0
                acc[6 + d] += __builtin_popcount((rt[i] ^ at[d]) & re[i] & ae[d]);  // ddy = +1
            }
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v += __shfl_xor(v, d);
    return v;
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

struct UnitPlan {
    int cw_log2, units_x, units;
};

__host__ __device__ __forceinline__ UnitPlan plan_level(const LevelGeom &lv, int rows)
{
    const int n32 = 2 * lv.wpr;
    int cw_log2 = 0;
    while ((1 << cw_log2) < n32 && cw_log2 < 6)
        ++cw_log2;
    UnitPlan p;
    p.cw_log2 = cw_log2;
    p.units_x = (n32 + (1 << cw_log2) - 1) >> cw_log2;
    const int rows_per_unit = rows * (kWave >> cw_log2);
    p.units = p.units_x * ((lv.h + rows_per_unit - 1) / rows_per_unit);
    return p;
}

__device__ __forceinline__ uint32_t load_counter(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run by the last workgroup to finish level 0: walks every pair's counters
// from the coarsest level down and writes the outputs.  Rows of images that
// are not the moving image of a pair (the reference) are zero.
__device__ void finalize(const SearchArgs &a)
{
    __shared__ uint32_t tot[kMaxStack][9];
    const int L = a.g.L;
    const SearchOutputs &o = a.out;
    for (int r = threadIdx.x; r < o.n_out; r += blockDim.x) {
        o.shifts[2 * r] = 0;
        o.shifts[2 * r + 1] = 0;
        o.errs[r] = 0u;
        if (o.trace)
            for (int i = 0; i < 9 * L; ++i)
                o.trace[(int64_t)r * 9 * L + i] = 0u;
        if (o.level_shifts)
            for (int i = 0; i < 2 * L; ++i)
                o.level_shifts[(int64_t)r * 2 * L + i] = 0;
    }
    __syncthreads();
    int bx = 0, by = 0, sx = 0, sy = 0;
    uint32_t err = 0;
    for (int l = L - 1; l >= 0; --l) {
        for (int i = threadIdx.x; i < a.npairs * 9; i += blockDim.x) {
            const int p = i / 9, c = i % 9;
            const uint32_t *cnt = a.state + (int64_t)p * a.state_stride + l * kCounterWords + c;
            uint32_t s = 0;
#pragma unroll
            for (int k = 0; k < kCopies; ++k)
                s += load_counter(cnt + 9 * k);
            tot[p][c] = s;
        }
        __syncthreads();
        if ((int)threadIdx.x < a.npairs) {
            const int p = threadIdx.x, r = o.pair_image[p];
            const int best = argmin9(tot[p]);
            sx = bx + best % 3 - 1;
            sy = by + best / 3 - 1;
            err = tot[p][best];
            if (o.trace)
                for (int i = 0; i < 9; ++i)
                    o.trace[((int64_t)r * L + l) * 9 + i] = tot[p][i];
            if (o.level_shifts) {
                o.level_shifts[((int64_t)r * L + l) * 2] = sx;
                o.level_shifts[((int64_t)r * L + l) * 2 + 1] = sy;
            }
            bx = 2 * sx;
            by = 2 * sy;
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < a.npairs) {
        const int r = o.pair_image[threadIdx.x];
        o.shifts[2 * r] = sx;
        o.shifts[2 * r + 1] = sy;
        o.errs[r] = err;
    }
}

// After this workgroup's counter updates: if it is the last workgroup of a
// launch that searched level 0, write the outputs.
//
// Ordering without device-wide fences (which on gfx950 write back the whole
// L2): the counters are only ever updated with agent-scope atomics and read
// back with agent-scope atomic loads, both performed at the coherence point.
// The workgroup barrier waits until this workgroup's counter atomics have
// completed before thread 0 takes its ticket, and the ticket counter is a
// single agent-scope atomic, so the workgroup that draws the last ticket
// observes every other workgroup's completed counter updates.
__device__ void finish_launch(const SearchArgs &a, int level)
{
    __shared__ int s_last;
    if (level != 0)
        return;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t nblocks = gridDim.x * gridDim.y;
        s_last = atomicAdd(a.done, 1u) == nblocks - 1;
    }
    __syncthreads();
    if (s_last)
        finalize(a);
}

// Levels L-1 .. coarse_lo of every pair, one 1024-thread workgroup per pair.
__global__ __launch_bounds__(1024) void k_search_coarse(SearchArgs a)
{
    __shared__ uint32_t red[16][9];
    __shared__ uint32_t tot[9];
    const int pair = blockIdx.x;
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    uint32_t *state = a.state + (int64_t)pair * a.state_stride;
    int32_t *bases = (int32_t *)(state + (int64_t)g.L * kCounterWords);
    int bx = 0, by = 0;
    for (int l = g.L - 1; l >= a.coarse_lo; --l) {
        const LevelGeom &lv = g.lv[l];
        const UnitPlan p = plan_level(lv, a.rows_per_stream);
        uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int u = wave; u < p.units; u += 16)
            search_unit(a.ref[pair], a.mov[pair], lv, bx, by, u, p.cw_log2, a.rows_per_stream, p.units_x, acc);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const uint32_t s = wave_sum(acc[i]);
            if (lane == 0)
                red[wave][i] = s;
        }
        __syncthreads();
        if (threadIdx.x < 9) {
            uint32_t s = 0;
            for (int w = 0; w < 16; ++w)
                s += red[w][threadIdx.x];
            tot[threadIdx.x] = s;
            state[l * kCounterWords + threadIdx.x] = s;  // copy 0 holds the total
        }
        __syncthreads();
        const int best = argmin9(tot);
        if (threadIdx.x == 0) {
            bases[2 * l] = bx;
            bases[2 * l + 1] = by;
        }
        bx = 2 * (bx + best % 3 - 1);
        by = 2 * (by + best / 3 - 1);
        __syncthreads();
    }
    finish_launch(a, a.coarse_lo);
}

// One large level of every pair: grid (workgroups per pair, pairs).
__global__ __launch_bounds__(256) void k_search_fine(SearchArgs a)
{
    __shared__ uint32_t cnt[kCounterWords];
    __shared__ int sbase[2];
    __shared__ uint32_t red[4][9];
    const int pair = blockIdx.y;
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    const int l = a.level;
    uint32_t *state = a.state + (int64_t)pair * a.state_stride;
    int32_t *bases = (int32_t *)(state + (int64_t)g.L * kCounterWords);

    // Base of this level = twice the winner of the level above.
    if (threadIdx.x < kCounterWords)
        cnt[threadIdx.x] = state[(l + 1) * kCounterWords + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c[9];
        for (int i = 0; i < 9; ++i) {
            uint32_t s = 0;
            for (int k = 0; k < kCopies; ++k)
                s += cnt[k * 9 + i];
            c[i] = s;
        }
        const int best = argmin9(c);
        sbase[0] = 2 * (bases[2 * (l + 1)] + best % 3 - 1);
        sbase[1] = 2 * (bases[2 * (l + 1) + 1] + best / 3 - 1);
        if (blockIdx.x == 0) {
            bases[2 * l] = sbase[0];
            bases[2 * l + 1] = sbase[1];
        }
    }
    __syncthreads();

    const LevelGeom &lv = g.lv[l];
    const UnitPlan p = plan_level(lv, a.rows_per_stream);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int unit = blockIdx.x * 4 + wave;
    if (unit < p.units)
        search_unit(a.ref[pair], a.mov[pair], lv, sbase[0], sbase[1], unit, p.cw_log2, a.rows_per_stream,
                    p.units_x, acc);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t s = wave_sum(acc[i]);
        if (lane == 0)
            red[wave][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const uint32_t s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                           red[3][threadIdx.x];
        if (s)
            atomicAdd(state + l * kCounterWords + (blockIdx.x % kCopies) * 9 + threadIdx.x, s);
    }
    finish_launch(a, l);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_zero(const ZeroArgs &a, hipStream_t s)
{
    if (a.count <= 0)
        return hipSuccess;
    int64_t most = 0;
    for (int i = 0; i < a.count; ++i)
        most = a.words[i] > most ? a.words[i] : most;
    int blocks = (int)((most + 255) / 256);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    {
        ProfScope prof_("k_zero", s);
        hipLaunchKernelGGL(k_zero, dim3(blocks, a.count), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_pyramid(const PyramidArgs &in, int cus, hipStream_t s)
{
    PyramidArgs a = in;
    a.tiles_x = (a.g.W + kTileW - 1) / kTileW;
    a.tiles_y = (a.g.H + kTileH - 1) / kTileH;
    const int64_t total = (int64_t)a.tiles_x * a.tiles_y * a.n;
    const int64_t want = (int64_t)cus * 4;
    int64_t per = (total + want - 1) / want;
    per = per < 1 ? 1 : per;
    a.tiles_per_block = (int32_t)per;
    const int blocks = (int)((total + per - 1) / per);
    {
        ProfScope prof_("k_pyramid", s);
        hipLaunchKernelGGL(k_pyramid, dim3(blocks), dim3(256), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.g.L <= kFused)
        return e;
    CoarsePyramidArgs c;
    for (int i = 0; i < a.n; ++i)
        c.pyr[i] = a.pyr[i];
    c.n = a.n;
    c.pad_ = 0;
    c.g = a.g;
    {
        ProfScope prof_("k_pyramid_coarse", s);
        hipLaunchKernelGGL(k_pyramid_coarse, dim3(a.n), dim3(256), 0, s, c);
    }
    return hipGetLastError();
}

hipError_t launch_bitmaps(const BitmapArgs &a, int cus, hipStream_t s)
{
    const int64_t total = a.chunk_start[a.g.L] * a.n;
    int64_t blocks = (total + 3) / 4;
    const int64_t cap = (int64_t)cus * 8;
    blocks = blocks > cap ? cap : (blocks < 1 ? 1 : blocks);
    {
        ProfScope prof_("k_bitmaps", s);
        hipLaunchKernelGGL(k_bitmaps, dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// Level sizes (in dwords) up to this many are searched by the single-workgroup
// coarse kernel; larger levels get a grid-wide launch each.
constexpr int64_t kCoarseDwords = 4096;

hipError_t launch_search(SearchArgs a, hipStream_t s)
{
    const Geometry &g = a.g;
    int lo = g.L;
    while (lo > 0 && (int64_t)2 * g.lv[lo - 1].wpr * g.lv[lo - 1].h <= kCoarseDwords)
        --lo;
    if (lo == g.L)
        lo = g.L - 1;  // the coarsest level always runs in the coarse kernel
    a.coarse_lo = lo;
    a.rows_per_stream = 4;
    {
        ProfScope prof_("k_search_coarse", s);
        hipLaunchKernelGGL(k_search_coarse, dim3(a.npairs), dim3(1024), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    for (int l = lo - 1; l >= 0; --l) {
        // 8 rows per stream, fewer when that leaves too few work units to fill the chip.
        int rows = 8;
        while (rows > 4 && (int64_t)plan_level(g.lv[l], rows).units * a.npairs < 4096)
            rows >>= 1;
        a.level = l;
        a.rows_per_stream = rows;
        const int blocks = (plan_level(g.lv[l], rows).units + 3) / 4;
        {
            ProfScope prof_("k_search_fine", s);
            hipLaunchKernelGGL(k_search_fine, dim3(blocks, a.npairs), dim3(256), 0, s, a);
        }
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace mtb
