// mtb_kernels.hip -- gfx950 kernels for MTB translational alignment.
//
// Pass 1  k_pyramid         RGB -> gray levels 0..6 of 64x64 tiles + LDS histograms
//         k_pyramid_coarse  levels 7.. from level 6 (one workgroup per image)
// Pass 2  k_bitmaps         gray -> lower median per level, packed T/E words
// Search  k_search_coarse   small levels, one workgroup per pair, all in one launch
//         k_search_fine     one launch per large level, grid over (units, pairs)
//         k_finalize        walks the per-level counters into shifts, errors, traces
//
// The arithmetic is integer throughout; reductions are integer adds, so the
// results do not depend on the order in which workgroups finish.

#include "mtb_internal.h"

namespace mtb {

namespace {

constexpr int kWave = 64;

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

// One 64x64 tile: 256 threads, each owns a 4x4 block of level-0 pixels.
// Levels 1 and 2 stay inside the thread, levels 3 and 4 combine lanes with
// cross-lane shuffles, levels 5 and 6 go through LDS.
__global__ __launch_bounds__(256) void k_pyramid(PyramidArgs a)
{
    __shared__ uint32_t hist[4][kFused][256];
    __shared__ uint32_t lvl4[2][4][4];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int bx = tid & 15, by = tid >> 4;
    const Geometry &g = a.g;
    const int fused = g.L < kFused ? g.L : kFused;

    for (int i = tid; i < 4 * kFused * 256; i += 256)
        (&hist[0][0][0])[i] = 0u;
    __syncthreads();

    const int64_t per_image = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t total = per_image * a.n;
    const int64_t t0 = (int64_t)blockIdx.x * a.tiles_per_block;
    const int64_t t1 = t0 + a.tiles_per_block < total ? t0 + a.tiles_per_block : total;

    auto flush = [&](int img) {
        __syncthreads();
        uint32_t *gh = (uint32_t *)(a.pyr[img] + g.hist_off);
        for (int l = 0; l < fused; ++l) {
            const uint32_t s = hist[0][l][tid] + hist[1][l][tid] + hist[2][l][tid] + hist[3][l][tid];
            hist[0][l][tid] = hist[1][l][tid] = hist[2][l][tid] = hist[3][l][tid] = 0u;
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
        const int X0 = tx * kTile, Y0 = ty * kTile;
        const int x0 = X0 + 4 * bx, y0 = Y0 + 4 * by;
        const uint8_t *rgb = a.rgb[img];
        uint8_t *pyr = a.pyr[img];

        // ---- level 0: gray of the 4x4 block
        uint32_t v[4][4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int y = y0 + rr;
            if (y < g.H && x0 < g.W) {
                const uint8_t *row = rgb + (int64_t)y * a.stride + 3 * (int64_t)x0;
                if (a.aligned && x0 + 3 < g.W) {
                    const uint32_t *p = (const uint32_t *)row;
                    const uint32_t d0 = p[0], d1 = p[1], d2 = p[2];
                    v[rr][0] = gray3(d0 & 255u, (d0 >> 8) & 255u, (d0 >> 16) & 255u);
                    v[rr][1] = gray3(d0 >> 24, d1 & 255u, (d1 >> 8) & 255u);
                    v[rr][2] = gray3((d1 >> 16) & 255u, d1 >> 24, d2 & 255u);
                    v[rr][3] = gray3((d2 >> 8) & 255u, (d2 >> 16) & 255u, d2 >> 24);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        v[rr][c] = (x0 + c < g.W) ? gray3(row[3 * c], row[3 * c + 1], row[3 * c + 2]) : 0u;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    v[rr][c] = 0u;
            }
        }
        {
            const LevelGeom &lv = g.lv[0];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int y = y0 + rr;
                if (y < g.H && x0 < g.W) {
                    // x0 < W <= pitch and pitch % 64 == 0, so all four bytes are inside the row.
                    *(uint32_t *)(pyr + lv.gray_off + (int64_t)y * lv.gray_pitch + x0) =
                        v[rr][0] | (v[rr][1] << 8) | (v[rr][2] << 16) | (v[rr][3] << 24);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (x0 + c < g.W)
                            atomicAdd(&hist[wave][0][v[rr][c]], 1u);
                }
            }
        }
        if (fused > 1) {
            // ---- level 1: 2x2 per thread
            uint32_t u1[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    u1[i][j] = (v[2 * i][2 * j] + v[2 * i][2 * j + 1] + v[2 * i + 1][2 * j] +
                                v[2 * i + 1][2 * j + 1]) >> 2;
            const LevelGeom &l1 = g.lv[1];
            const int x1 = x0 >> 1, y1 = y0 >> 1;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (y1 + i < l1.h && x1 < l1.w) {
                    *(uint16_t *)(pyr + l1.gray_off + (int64_t)(y1 + i) * l1.gray_pitch + x1) =
                        (uint16_t)(u1[i][0] | (u1[i][1] << 8));
                    atomicAdd(&hist[wave][1][u1[i][0]], 1u);
                    if (x1 + 1 < l1.w)
                        atomicAdd(&hist[wave][1][u1[i][1]], 1u);
                }
            }
            if (fused > 2) {
                // ---- level 2: 1 pixel per thread
                const uint32_t u2 = (u1[0][0] + u1[0][1] + u1[1][0] + u1[1][1]) >> 2;
                const LevelGeom &l2 = g.lv[2];
                const int x2 = x0 >> 2, y2 = y0 >> 2;
                if (x2 < l2.w && y2 < l2.h) {
                    pyr[l2.gray_off + (int64_t)y2 * l2.gray_pitch + x2] = (uint8_t)u2;
                    atomicAdd(&hist[wave][2][u2], 1u);
                }
                if (fused > 3) {
                    // ---- level 3: 2x2 threads (lane ^ 1 is bx ^ 1, lane ^ 16 is by ^ 1)
                    uint32_t s3 = u2 + __shfl_xor(u2, 1);
                    s3 += __shfl_xor(s3, 16);
                    const uint32_t u3 = s3 >> 2;
                    const LevelGeom &l3 = g.lv[3];
                    const int x3 = x0 >> 3, y3 = y0 >> 3;
                    if (((bx | by) & 1) == 0 && x3 < l3.w && y3 < l3.h) {
                        pyr[l3.gray_off + (int64_t)y3 * l3.gray_pitch + x3] = (uint8_t)u3;
                        atomicAdd(&hist[wave][3][u3], 1u);
                    }
                    if (fused > 4) {
                        // ---- level 4: lane ^ 2 is bx ^ 2, lane ^ 32 is by ^ 2 (same wave)
                        uint32_t s4 = u3 + __shfl_xor(u3, 2);
                        s4 += __shfl_xor(s4, 32);
                        const uint32_t u4 = s4 >> 2;
                        const LevelGeom &l4 = g.lv[4];
                        const int x4 = x0 >> 4, y4 = y0 >> 4;
                        const bool own4 = ((bx | by) & 3) == 0;
                        if (own4 && x4 < l4.w && y4 < l4.h) {
                            pyr[l4.gray_off + (int64_t)y4 * l4.gray_pitch + x4] = (uint8_t)u4;
                            atomicAdd(&hist[wave][4][u4], 1u);
                        }
                        if (fused > 5) {
                            // ---- levels 5 and 6 through LDS: the tile has 4x4 level-4 pixels,
                            // row = wave, column = bx / 4.
                            if (own4)
                                lvl4[parity][wave][bx >> 2] = u4;
                            __syncthreads();
                            if (tid < 4) {
                                const int i5 = tid >> 1, j5 = tid & 1;
                                const uint32_t(*q)[4] = lvl4[parity];
                                const uint32_t u5 = (q[2 * i5][2 * j5] + q[2 * i5][2 * j5 + 1] +
                                                     q[2 * i5 + 1][2 * j5] + q[2 * i5 + 1][2 * j5 + 1]) >> 2;
                                const LevelGeom &l5 = g.lv[5];
                                const int x5 = (X0 >> 5) + j5, y5 = (Y0 >> 5) + i5;
                                if (x5 < l5.w && y5 < l5.h) {
                                    pyr[l5.gray_off + (int64_t)y5 * l5.gray_pitch + x5] = (uint8_t)u5;
                                    atomicAdd(&hist[0][5][u5], 1u);
                                }
                                if (fused > 6 && tid == 0) {
                                    uint32_t s6 = 0;
#pragma unroll
                                    for (int i = 0; i < 2; ++i)
#pragma unroll
                                        for (int j = 0; j < 2; ++j)
                                            s6 += (q[2 * i][2 * j] + q[2 * i][2 * j + 1] + q[2 * i + 1][2 * j] +
                                                   q[2 * i + 1][2 * j + 1]) >> 2;
                                    const uint32_t u6 = s6 >> 2;
                                    const LevelGeom &l6 = g.lv[6];
                                    const int x6 = X0 >> 6, y6 = Y0 >> 6;
                                    if (x6 < l6.w && y6 < l6.h) {
                                        pyr[l6.gray_off + (int64_t)y6 * l6.gray_pitch + x6] = (uint8_t)u6;
                                        atomicAdd(&hist[0][6][u6], 1u);
                                    }
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
    const uint64_t hit = __ballot(incl >= need);
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

// Each wavefront takes chunks of kChunkWords consecutive 64-pixel words of
// one level: 16 bytes of gray per lane, transposed through LDS so that lane i
// holds pixel i of each word; a ballot then yields the word directly.
__global__ __launch_bounds__(256) void k_bitmaps(BitmapArgs a)
{
    __shared__ uint4 stage[4][kWave];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    const int64_t per_image = a.chunk_start[g.L];
    const int64_t total = per_image * a.n;
    const uint32_t X = (uint32_t)a.exclude;
    const uint8_t *st = (const uint8_t *)&stage[wave][0];

    int cur_img = -1, cur_l = -1;
    uint32_t m = 0;
    for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < total; c += (int64_t)gridDim.x * 4) {
        const int img = (int)(c / per_image);
        const int64_t cc = c - (int64_t)img * per_image;
        int l = 0;
        while (cc >= a.chunk_start[l + 1])
            ++l;
        const LevelGeom &lv = g.lv[l];
        if (img != cur_img || l != cur_l) {
            m = wave_median((const uint32_t *)(a.pyr[img] + g.hist_off) + 256 * l, (uint32_t)(lv.w * lv.h));
            cur_img = img;
            cur_l = l;
        }
        const int w0 = (int)(cc - a.chunk_start[l]) * kChunkWords;
        const int nwords = lv.h * lv.wpr;
        const int cnt = nwords - w0 < kChunkWords ? nwords - w0 : kChunkWords;
        if (w0 == 0 && lane == 0)
            ((int32_t *)(a.bm[img] + g.med_off))[l] = (int32_t)m;

        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (lane * 16 < cnt * 64)
            v = *(const uint4 *)(a.pyr[img] + lv.gray_off + (int64_t)w0 * 64 + lane * 16);
        __builtin_amdgcn_wave_barrier();
        stage[wave][lane] = v;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        uint64_t my_t = 0, my_e = 0;
        int k = w0 % lv.wpr;  // word index within its row
        for (int j = 0; j < cnt; ++j) {
            const uint32_t gv = st[j * 64 + lane];
            const bool valid = k * 64 + lane < lv.w;
            const uint64_t tw = __ballot(valid && gv > m);
            const uint64_t ew = __ballot(valid && (gv - m + X) > 2u * X);
            if (lane == j)
                my_t = tw;
            if (lane == 16 + j)
                my_e = ew;
            if (++k == lv.wpr)
                k = 0;
        }
        uint64_t *tb = (uint64_t *)(a.bm[img] + lv.tb_off);
        uint64_t *eb = (uint64_t *)(a.bm[img] + lv.eb_off);
        if (lane < cnt)
            tb[w0 + lane] = my_t;
        else if (lane >= 16 && lane - 16 < cnt)
            eb[w0 + lane - 16] = my_e;
    }
}

// ---------------------------------------------------------------- search

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// The three horizontally shifted copies (ddx = -1, 0, +1 -> index 0, 1, 2) of
// one 32-pixel word of a moving bitmap row, for column k and base shift bx.
// Bits [t, t+32) of the row with t = 32k - (bx + ddx); words outside the row
// and rows outside the level read as 0 (zero fill).
struct Shifted {
    uint32_t t[3], e[3];
};

__device__ __forceinline__ Shifted moving_row(const uint32_t *tm, const uint32_t *em, int j, int h,
                                              int n32, int q, uint32_t r)
{
    uint32_t t0 = 0, t1 = 0, t2 = 0, e0 = 0, e1 = 0, e2 = 0;
    if (j >= 0 && j < h) {
        const uint32_t *pt = tm + j * n32;
        const uint32_t *pe = em + j * n32;
        if (q >= 0 && q < n32) {
            t0 = pt[q];
            e0 = pe[q];
        }
        if (q + 1 >= 0 && q + 1 < n32) {
            t1 = pt[q + 1];
            e1 = pe[q + 1];
        }
        if (q + 2 >= 0 && q + 2 < n32) {
            t2 = pt[q + 2];
            e2 = pe[q + 2];
        }
    }
    Shifted s;
    s.t[2] = funnel(t1, t0, r);
    s.e[2] = funnel(e1, e0, r);
    if (r + 1 < 32) {
        s.t[1] = funnel(t1, t0, r + 1);
        s.e[1] = funnel(e1, e0, r + 1);
    } else {
        s.t[1] = t1;
        s.e[1] = e1;
    }
    if (r + 2 < 32) {
        s.t[0] = funnel(t1, t0, r + 2);
        s.e[0] = funnel(e1, e0, r + 2);
    } else {
        s.t[0] = funnel(t2, t1, r + 2 - 32);
        s.e[0] = funnel(e2, e1, r + 2 - 32);
    }
    return s;
}

__device__ __forceinline__ void score_row(uint32_t tr, uint32_t er, const Shifted &s, uint32_t *acc)
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        acc[d] += __builtin_popcount((tr ^ s.t[d]) & er & s.e[d]);
}

// Nine candidate errors of one work unit: a wavefront covers CW = 2^cw_log2
// dword columns and 64 / CW row streams of rows_per_unit rows each.
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

    // Rows of the moving image seen by reference row y: y - by - ddy.
    Shifted a = moving_row(tm, em, y_begin - by - 1, h, n32, q, r);  // ddy = +1
    Shifted b = moving_row(tm, em, y_begin - by, h, n32, q, r);      // ddy = 0
    for (int y = y_begin; y < y_end; ++y) {
        const Shifted c = moving_row(tm, em, y - by + 1, h, n32, q, r);  // ddy = -1
        uint32_t t = 0, e = 0;
        if (col_ok) {
            t = tr[y * n32 + k];
            e = er[y * n32 + k];
        }
        score_row(t, e, c, acc + 0);
        score_row(t, e, b, acc + 3);
        score_row(t, e, a, acc + 6);
        a = b;
        b = c;
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
    int cw_log2, rows, units_x, units;
};

__device__ __forceinline__ UnitPlan plan_level(const LevelGeom &lv, int rows)
{
    const int n32 = 2 * lv.wpr;
    int cw_log2 = 0;
    while ((1 << cw_log2) < n32 && cw_log2 < 6)
        ++cw_log2;
    UnitPlan p;
    p.cw_log2 = cw_log2;
    p.rows = rows;
    p.units_x = (n32 + (1 << cw_log2) - 1) >> cw_log2;
    const int rows_per_unit = rows * (kWave >> cw_log2);
    p.units = p.units_x * ((lv.h + rows_per_unit - 1) / rows_per_unit);
    return p;
}

// Levels L-1 .. coarse_lo of every pair, one 1024-thread workgroup per pair.
__global__ __launch_bounds__(1024) void k_search_coarse(SearchArgs a)
{
    __shared__ uint32_t red[16][9];
    __shared__ uint32_t tot[9];
    const int pair = blockIdx.x;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const Geometry &g = a.g;
    uint32_t *state = a.state + (int64_t)pair * a.state_stride;
    int32_t *bases = (int32_t *)(state + (int64_t)g.L * kCounterWords);
    int bx = 0, by = 0;
    for (int l = g.L - 1; l >= a.coarse_lo; --l) {
        const LevelGeom &lv = g.lv[l];
        const UnitPlan p = plan_level(lv, a.rows_per_unit);
        uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int u = wave; u < p.units; u += 16)
            search_unit(a.ref[pair], a.mov[pair], lv, bx, by, u, p.cw_log2, p.rows, p.units_x, acc);
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
}

// One large level of every pair: grid (workgroups per pair, pairs).
__global__ __launch_bounds__(256) void k_search_fine(SearchArgs a)
{
    __shared__ uint32_t cnt[kCounterWords];
    __shared__ int sbase[2];
    __shared__ uint32_t red[4][9];
    const int pair = blockIdx.y;
    const int wave = threadIdx.x >> 6;
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
    const UnitPlan p = plan_level(lv, a.rows_per_unit);
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int unit = blockIdx.x * 4 + wave;
    if (unit < p.units)
        search_unit(a.ref[pair], a.mov[pair], lv, sbase[0], sbase[1], unit, p.cw_log2, p.rows,
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
}

// Walks every pair's counters from the coarsest level down and writes the
// outputs; rows of images that are not the moving image of a pair are zero.
__global__ __launch_bounds__(64) void k_finalize(FinalizeArgs a)
{
    const int L = a.L;
    for (int o = threadIdx.x; o < a.n_out; o += blockDim.x) {
        a.shifts[2 * o] = 0;
        a.shifts[2 * o + 1] = 0;
        a.errs[o] = 0u;
        if (a.trace)
            for (int i = 0; i < 9 * L; ++i)
                a.trace[(int64_t)o * 9 * L + i] = 0u;
        if (a.level_shifts)
            for (int i = 0; i < 2 * L; ++i)
                a.level_shifts[(int64_t)o * 2 * L + i] = 0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < a.npairs; p += blockDim.x) {
        const uint32_t *state = a.state + (int64_t)p * a.state_stride;
        const int o = a.pair_image[p];
        int bx = 0, by = 0, sx = 0, sy = 0;
        uint32_t err = 0;
        for (int l = L - 1; l >= 0; --l) {
            uint32_t c[9];
            for (int i = 0; i < 9; ++i) {
                uint32_t s = 0;
                for (int k = 0; k < kCopies; ++k)
                    s += state[l * kCounterWords + k * 9 + i];
                c[i] = s;
            }
            const int best = argmin9(c);
            sx = bx + best % 3 - 1;
            sy = by + best / 3 - 1;
            err = c[best];
            if (a.trace)
                for (int i = 0; i < 9; ++i)
                    a.trace[((int64_t)o * L + l) * 9 + i] = c[i];
            if (a.level_shifts) {
                a.level_shifts[((int64_t)o * L + l) * 2] = sx;
                a.level_shifts[((int64_t)o * L + l) * 2 + 1] = sy;
            }
            bx = 2 * sx;
            by = 2 * sy;
        }
        a.shifts[2 * o] = sx;
        a.shifts[2 * o + 1] = sy;
        a.errs[o] = err;
    }
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

hipError_t launch_search(SearchArgs a, int /*unused*/, hipStream_t s)
{
    const Geometry &g = a.g;
    int lo = g.L;
    while (lo > 0 && (int64_t)2 * g.lv[lo - 1].wpr * g.lv[lo - 1].h <= kCoarseDwords)
        --lo;
    if (lo == g.L)
        lo = g.L - 1;  // the coarsest level always runs in the coarse kernel
    a.coarse_lo = lo;
    a.rows_per_unit = 4;
    {
        ProfScope prof_("k_search_coarse", s);
        hipLaunchKernelGGL(k_search_coarse, dim3(a.npairs), dim3(1024), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    for (int l = lo - 1; l >= 0; --l) {
        const LevelGeom &lv = g.lv[l];
        const int n32 = 2 * lv.wpr;
        int cw_log2 = 0;
        while ((1 << cw_log2) < n32 && cw_log2 < 6)
            ++cw_log2;
        const int units_x = (n32 + (1 << cw_log2) - 1) >> cw_log2;
        const int streams = kWave >> cw_log2;
        // About 16 rows per stream, fewer when that leaves too few work units.
        int rows = 16;
        const int64_t target_units = 2048;
        while (rows > 2 && (int64_t)units_x * ((lv.h + rows * streams - 1) / (rows * streams)) * a.npairs <
                               target_units)
            rows >>= 1;
        a.level = l;
        a.rows_per_unit = rows;
        const int units = units_x * ((lv.h + rows * streams - 1) / (rows * streams));
        const int blocks = (units + 3) / 4;
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

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s)
{
    {
        ProfScope prof_("k_finalize", s);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace mtb
