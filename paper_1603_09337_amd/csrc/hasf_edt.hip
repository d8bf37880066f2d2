// Exact squared Euclidean distance transform on gfx950 (Sec. 4.1).
//
// The transform is separable: d2(i, j) = min_k (j - k)^2 + g(i, k)^2 where
// g(i, k) is the distance from row i to the nearest feature of column k
// (phase 1, columns; phase 2, rows). The paper's CPU version deals whole
// columns and whole rows to threads; a column scan is sequential in rows, so
// here phase 1 is split into 32-row segments that are independent:
//
//   edt_colmask   one thread per 4 columns and 32-row segment: the segment's
//                 features as 32-bit masks (reads the input once, 4 bytes per
//                 load).
//   edt_colcarry  16 threads per column: for every segment, the nearest
//                 feature row above the segment and below it (a prefix-max /
//                 suffix-min over the segment masks, in 16 chunks combined
//                 through LDS; with at most 8 segments per chunk the masks
//                 stay in registers between the scan and the writes).
//   edt_rows32    one workgroup per strip of rows: g^2 of the strip from the
//                 masks and carries (O(1) per pixel with clz/ctz), kept in
//                 LDS as uint32 with "infinity" columns padding each row,
//                 then phase 2 per pixel as an exact windowed minimum:
//                 starting from g(i, j)^2, columns j -+ 1, j -+ 2, ... are
//                 visited until d^2 reaches the best value found, beyond which
//                 no column can improve it. Within the padding a candidate
//                 costs one saturating add and one min; the result is
//                 written once. edt_rows is the same with uint16 g, for rows
//                 too wide for a uint32 strip in LDS.
//   edt_rows_env  the windowed search costs each pixel about its distance to
//                 the nearest feature, so a strip whose column distances
//                 average more than ENV_AVG and whose searches, sampled at
//                 one pixel per thread, are long too is instead listed by
//                 edt_rows32 and done here, one row per workgroup, with Alg. 2's lower
//                 envelope built in parallel: the lower convex hull of the
//                 points (k, k^2 + g(k)^2) per band of columns (a stack per
//                 thread), the bands' hulls merged pairwise in log rounds
//                 (common lower tangents), then each thread's pixels read
//                 off the hull by bisection and a forward walk. Its cost
//                 does not depend on the distances; the frame is applied
//                 as a minimum at the end, so sparse rows keep small hulls.
//                 g is finite exactly in the columns that hold a feature
//                 somewhere, so every row has the same such columns
//                 (edt_colcarry marks and counts them); when there are at
//                 most ENV_FEW, edt_rows32 leaves every row to edt_rows_env
//                 unread, and each row takes the minimum over them directly
//                 (each thread a run of consecutive pixels, whose lowest
//                 column only moves right).
//
// HBM traffic: 1 B/px read + 4 B/px written, plus 3/8 B/px of masks and
// carries; the per-column g never leaves LDS. With no feature at all (and no
// frame) every column is empty, which the strip kernel sees by itself.
#include <algorithm>
#include <atomic>
#include <mutex>

#include "hasf_common.h"

namespace {

constexpr int SEG = 32;
constexpr uint16_t G_INF = 0xFFFF;
constexpr uint32_t G2_INF = 0xFFFFFFFFu;
constexpr int ROWS_BLOCK = 1024;
constexpr int PAD = 16;  // "infinity" columns on each side of a uint32 strip row
constexpr int NO_ROW_BELOW = 0x7FFFFFFF;
constexpr int CARRY_GROUPS = 16;  // threads per column in edt_colcarry
constexpr int CARRY_COLS = 16;    // columns per edt_colcarry workgroup
constexpr int CARRY_REG = 8;      // segments per thread kept in registers by edt_colcarry
// A strip goes to edt_rows_env when its pixels' column distances, each
// counted up to ENV_CAP (a column with no feature counts ENV_CAP), average
// more than ENV_AVG: the windowed search costs a pixel about its distance.
constexpr int ENV_AVG = 16;
constexpr int ENV_CAP = 1024;
// The column distances overstate the search where features are scattered
// (a pixel's nearest feature is then much nearer than the nearest in its own
// column), so a strip over ENV_AVG is listed only when a sample of its
// searches (one pixel per thread, each stopped at SAMPLE_MAX columns and then
// counted as ENV_CAP) averages more than SAMPLE_AVG columns.
constexpr int SAMPLE_MAX = 64;
constexpr int SAMPLE_AVG = 64;
constexpr int ENV_NT = 256;       // threads of an edt_rows_env workgroup (one row at a time)
constexpr int ENV_W_MAX = 16384;  // widest row edt_rows_env takes (its LDS: about 8 bytes per column)
// an image with at most this many columns that hold a feature: edt_rows_env
// takes the minimum over those columns directly
constexpr int ENV_FEW = 32;
// the columns with a feature are counted in FC_PARTS counters (a workgroup
// of edt_colcarry adds to counter blockIdx.x % FC_PARTS), FC_STRIDE ints
// apart, so that few atomics queue on each, and FC_BASE ints after the count
// of listed strips, so that reading them does not slow the listing's
// atomics (measured: with the counters in the strip count's 512 bytes, the
// listing of 2048 strips took 40 us longer)
constexpr int FC_PARTS = 8;
constexpr int FC_STRIDE = 16;
constexpr int FC_BASE = 1024;
constexpr int CTL_INTS = FC_BASE + FC_STRIDE * FC_PARTS;  // the strip count and the counters

__device__ __forceinline__ int fc_index(int x)  // counter x = 0 .. FC_PARTS - 1
{
    return FC_BASE + x * FC_STRIDE;
}

__device__ __forceinline__ int feature_columns(const int* __restrict__ ctl)
{
    int n = 0;
#pragma unroll
    for (int x = 0; x < FC_PARTS; ++x)
        n += ctl[fc_index(x)];
    return n;
}
static_assert(ENV_FEW <= 64, "the feature columns are sorted and evaluated by one wave");

// one thread per 4 columns and 32-row segment: the segment's features as masks
__global__ __launch_bounds__(256) void edt_colmask(const uint8_t* __restrict__ F, long long ld, int H, int W,
                                                   int invert, int vec4, uint32_t* __restrict__ mask,
                                                   int* __restrict__ hard_count)
{
    const int c4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const int s = blockIdx.y;
    // the list of strips for edt_rows_env and the count of columns with a
    // feature start empty (this kernel runs first)
    if (hard_count && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x <= FC_PARTS)
        hard_count[threadIdx.x == 0 ? 0 : fc_index((int)threadIdx.x - 1)] = 0;
    if (c4 >= W)
        return;
    const int r0 = s * SEG;
    const int n = min(SEG, H - r0);
    const uint32_t valid = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    const uint32_t flip = invert ? valid : 0u;
    const uint8_t* p = F + (long long)r0 * ld + c4;
    if (vec4 && c4 + 4 <= W) {
        uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
#pragma unroll 8
        for (int b = 0; b < n; ++b) {
            const uint32_t v = *reinterpret_cast<const uint32_t*>(p + (long long)b * ld);
            m0 |= (uint32_t)((v & 0xFFu) != 0) << b;
            m1 |= (uint32_t)((v & 0xFF00u) != 0) << b;
            m2 |= (uint32_t)((v & 0xFF0000u) != 0) << b;
            m3 |= (uint32_t)((v & 0xFF000000u) != 0) << b;
        }
        uint32_t* out = mask + (size_t)s * W + c4;
        out[0] = m0 ^ flip;
        out[1] = m1 ^ flip;
        out[2] = m2 ^ flip;
        out[3] = m3 ^ flip;
        return;
    }
    for (int c = c4; c < min(c4 + 4, W); ++c) {
        uint32_t m = 0;
        for (int b = 0; b < n; ++b)
            m |= (uint32_t)(p[(long long)b * ld + (c - c4)] != 0) << b;
        mask[(size_t)s * W + c] = m ^ flip;
    }
}

// Per column and segment: the nearest feature row above the segment
// (above, -1 if none) and below it (below, NO_ROW_BELOW if none). A block
// covers CARRY_COLS columns; the CARRY_GROUPS threads of a column split its
// segments into consecutive groups, scan them, and combine through LDS.
//
// fcb, fcn (may be NULL): bit l of fcb[blockIdx.x] says whether column
// blockIdx.x * CARRY_COLS + l holds a feature, and the counters of fcn
// (see feature_columns) count such columns (stores and an atomic that
// nothing waits for).
__device__ __forceinline__ void note_feature_columns(const int (*glast)[CARRY_COLS], int c, int W,
                                                     uint16_t* __restrict__ fcb, int* __restrict__ fcn)
{
    // called by all of wave 0; lanes 0 .. CARRY_COLS - 1 stand for the
    // workgroup's columns (c is lane lc's column)
    const int lc = threadIdx.x;
    bool has = false;
    if (lc < CARRY_COLS && c < W)
        for (int k = 0; k < CARRY_GROUPS; ++k)
            has |= glast[k][lc] >= 0;
    const uint64_t bal = __ballot(has);
    if (lc == 0) {
        fcb[blockIdx.x] = (uint16_t)bal;
        if (bal)
            atomicAdd(fcn + fc_index(blockIdx.x % FC_PARTS), (int)__popcll(bal));
    }
}

__global__ __launch_bounds__(CARRY_COLS* CARRY_GROUPS) void edt_colcarry(const uint32_t* __restrict__ mask,
                                                                         int nseg, int W,
                                                                         int* __restrict__ above,
                                                                         int* __restrict__ below,
                                                                         uint16_t* __restrict__ fcb,
                                                                         int* __restrict__ fcn)
{
    static_assert(CARRY_COLS <= 16, "one 16-bit word of feature columns per workgroup");
    __shared__ int glast[CARRY_GROUPS][CARRY_COLS], gfirst[CARRY_GROUPS][CARRY_COLS];
    const int lc = threadIdx.x % CARRY_COLS, grp = threadIdx.x / CARRY_COLS;
    const int c = blockIdx.x * CARRY_COLS + lc;
    const int G = (nseg + CARRY_GROUPS - 1) / CARRY_GROUPS;
    const int s0 = grp * G, s1 = min(nseg, s0 + G);
    int last = -1, first = NO_ROW_BELOW;
    if (G <= CARRY_REG) {
        // few segments per thread (H <= CARRY_REG * CARRY_GROUPS * 32): the
        // masks stay in registers for the two writing passes
        uint32_t mr[CARRY_REG];
#pragma unroll
        for (int k = 0; k < CARRY_REG; ++k)
            mr[k] = (c < W && s0 + k < s1) ? mask[(size_t)(s0 + k) * W + c] : 0u;
#pragma unroll
        for (int k = 0; k < CARRY_REG; ++k)
            if (mr[k]) {
                last = (s0 + k) * SEG + 31 - __clz(mr[k]);
                if (first == NO_ROW_BELOW)
                    first = (s0 + k) * SEG + __ffs(mr[k]) - 1;
            }
        glast[grp][lc] = last;
        gfirst[grp][lc] = first;
        __syncthreads();
        if (fcb && threadIdx.x < 64)
            note_feature_columns(glast, c, W, fcb, fcn);
        if (c >= W)
            return;
        int up = -1, dn = NO_ROW_BELOW;
        for (int k = 0; k < grp; ++k)
            up = max(up, glast[k][lc]);
        for (int k = CARRY_GROUPS - 1; k > grp; --k)
            dn = min(dn, gfirst[k][lc]);
#pragma unroll
        for (int k = 0; k < CARRY_REG; ++k) {
            if (s0 + k >= s1)
                break;
            above[(size_t)(s0 + k) * W + c] = up;
            if (mr[k])
                up = (s0 + k) * SEG + 31 - __clz(mr[k]);
        }
#pragma unroll
        for (int k = CARRY_REG - 1; k >= 0; --k) {
            if (s0 + k >= s1)
                continue;
            below[(size_t)(s0 + k) * W + c] = dn;
            if (mr[k])
                dn = (s0 + k) * SEG + __ffs(mr[k]) - 1;
        }
        return;
    }
    if (c < W) {
#pragma unroll 8
        for (int s = s0; s < s1; ++s) {
            const uint32_t m = mask[(size_t)s * W + c];
            if (m) {
                last = s * SEG + 31 - __clz(m);
                if (first == NO_ROW_BELOW)
                    first = s * SEG + __ffs(m) - 1;
            }
        }
    }
    glast[grp][lc] = last;
    gfirst[grp][lc] = first;
    __syncthreads();
    if (fcb && threadIdx.x < 64)
        note_feature_columns(glast, c, W, fcb, fcn);
    if (c >= W)
        return;
    int up = -1, dn = NO_ROW_BELOW;
    for (int k = 0; k < grp; ++k)
        up = max(up, glast[k][lc]);
    for (int k = CARRY_GROUPS - 1; k > grp; --k)
        dn = min(dn, gfirst[k][lc]);
#pragma unroll 8
    for (int s = s0; s < s1; ++s) {
        above[(size_t)s * W + c] = up;
        const uint32_t m = mask[(size_t)s * W + c];
        if (m)
            up = s * SEG + 31 - __clz(m);
    }
#pragma unroll 8
    for (int s = s1 - 1; s >= s0; --s) {
        below[(size_t)s * W + c] = dn;
        const uint32_t m = mask[(size_t)s * W + c];
        if (m)
            dn = s * SEG + __ffs(m) - 1;
    }
}

// One workgroup per strip of `strip` rows (strip divides 32, so a strip lies
// in one segment): g of the strip into LDS (per column: the segment's mask
// and carries, then clz/ctz per row), then the exact row minimum per pixel.
__global__ __launch_bounds__(ROWS_BLOCK) void edt_rows(const uint32_t* __restrict__ mask,
                                                       const int* __restrict__ above,
                                                       const int* __restrict__ below, int H, int W,
                                                       int frame, int strip, uint32_t* __restrict__ d2, long long ldo)
{
    extern __shared__ uint16_t gs[];
    const int r0 = blockIdx.x * strip;
    const int nr = min(strip, H - r0);
    const int s = r0 / SEG;
    int has = 0;
    for (int c = threadIdx.x; c < W; c += blockDim.x) {
        const uint32_t m = mask[(size_t)s * W + c];
        const int up0 = above[(size_t)s * W + c];
        const int dn0 = below[(size_t)s * W + c];
        has |= (m != 0) | (up0 >= 0) | (dn0 != NO_ROW_BELOW);
        for (int r = 0; r < nr; ++r) {
            const int i = r0 + r;
            const int b = i - s * SEG;
            const uint32_t lo = m & (0xFFFFFFFFu >> (31 - b));  // rows <= i in the segment
            const uint32_t hi = m >> b;                         // rows >= i
            const int up = lo ? s * SEG + 31 - __clz(lo) : up0;
            const int dn = hi ? i + __ffs(hi) - 1 : dn0;
            int g = NO_ROW_BELOW;
            if (up >= 0)
                g = i - up;
            if (dn != NO_ROW_BELOW)
                g = min(g, dn - i);
            if (frame)
                g = min(g, min(i + 1, H - i));
            gs[r * W + c] = g == NO_ROW_BELOW ? G_INF : (uint16_t)g;
        }
    }
    // a column either has a feature somewhere or none: if no column has one,
    // the feature set is empty
    const int any = __syncthreads_or(has);
    if (!frame && !any) {
        for (int r = 0; r < nr; ++r)
            for (int j = threadIdx.x; j < W; j += blockDim.x)
                d2[(long long)(r0 + r) * ldo + j] = 0xFFFFFFFFu;
        return;
    }
    // per pixel, exact minimum over columns by increasing |j - k|: stop when
    // (j - k)^2 alone reaches the best value found
    for (int r = 0; r < nr; ++r) {
        const uint16_t* gr = gs + r * W;
        for (int j = threadIdx.x; j < W; j += blockDim.x) {
            const uint32_t g0 = gr[j];
            uint32_t best = g0 == G_INF ? 0xFFFFFFFFu : g0 * g0;
            if (frame) {
                const uint32_t e = (uint32_t)min(j + 1, W - j);
                best = min(best, e * e);
            }
            // four columns per side per step, loads issued together; columns
            // past the stopping point cannot improve best
            for (int d0 = 1;; d0 += 4) {
                if ((uint32_t)d0 * (uint32_t)d0 >= best || (j - d0 < 0 && j + d0 >= W))
                    break;
                uint32_t gl[4], gg[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int d = d0 + u;
                    gl[u] = j - d >= 0 ? gr[j - d] : G_INF;
                    gg[u] = j + d < W ? gr[j + d] : G_INF;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t dd = (uint32_t)(d0 + u) * (uint32_t)(d0 + u);
                    if (gl[u] != G_INF)
                        best = min(best, dd + gl[u] * gl[u]);
                    if (gg[u] != G_INF)
                        best = min(best, dd + gg[u] * gg[u]);
                }
            }
            d2[(long long)(r0 + r) * ldo + j] = best;
        }
    }
}

// Phase 2 for column j of one row: min over k of (j - k)^2 + g2[k], where
// gr points at the row's first column and has PAD columns of padding on each
// side (G2_INF, or 0 with the frame). Columns are visited by increasing
// |j - k| until (j - k)^2 alone reaches the best value found, beyond which no
// column can improve it.
__device__ __forceinline__ uint32_t row_min(const uint32_t* gr, int j, int W, int frame)
{
    uint32_t best = gr[j];
    // d = 1 .. PAD, four per step, no bounds checks (with the frame, the zero
    // padding supplies the distance to the left and right frame when it is
    // within PAD columns)
    int d = 1;
#pragma unroll
    for (int step = 0; step < PAD / 4; ++step) {
        const int d0 = 1 + 4 * step;
        if ((uint32_t)(d0 * d0) >= best)
            break;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t dd = (uint32_t)((d0 + u) * (d0 + u));
            best = min(best, __builtin_elementwise_add_sat(dd, gr[j - d0 - u]));
            best = min(best, __builtin_elementwise_add_sat(dd, gr[j + d0 + u]));
        }
        d = d0 + 4;
    }
    // beyond the padding: with bounds checks (a uint32 strip row fits LDS
    // only for W < 41000, so d + 3 and e stay below 2^16 and the 24-bit
    // multiplies are exact)
    if (frame && __umul24(d, d) < best) {
        const uint32_t e = (uint32_t)min(j + 1, W - j);
        best = min(best, __umul24(e, e));
    }
    // four columns a side per step, as within the padding (columns past the
    // point where the search could stop are real candidates too, so they
    // leave the minimum exact)
    for (; __umul24(d, d) < best && (j - d >= 0 || j + d < W); d += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t dd = __umul24(d + u, d + u);
            if (j - d - u >= 0)
                best = min(best, __builtin_elementwise_add_sat(dd, gr[j - d - u]));
            if (j + d + u < W)
                best = min(best, __builtin_elementwise_add_sat(dd, gr[j + d + u]));
        }
    }
    return best;
}

// Columns row_min would visit at one pixel of the strip (the distance at
// which its search ends, to four columns), or ENV_CAP when that is
// SAMPLE_MAX or more. Thread t of the first per * nr takes row t % nr and
// column k * s + r mod W (k = t / nr, s = (W / per) | 1): an odd stride, so
// the lanes of a wave read different LDS banks. Out of line: it runs only for strips the column
// distances would list, and inlined it costs the strip kernel's common case.
__device__ __attribute__((noinline)) uint32_t search_len(const uint32_t* g2s, int WP, int nr, int per, int W,
                                                         int frame)
{
    const int t = (int)threadIdx.x;
    if (t >= per * nr)
        return 0;
    const int r = t % nr, k = t / nr;
    const int j = (int)(((long long)k * ((W / per) | 1) + r) % W);
    const uint32_t* gr = g2s + r * WP + PAD;
    uint32_t best = gr[j];
    if (frame) {
        const uint32_t e = (uint32_t)min(j + 1, W - j);
        best = min(best, __umul24(e, e));
    }
    // four columns a side per step (the end is tested once per step, so
    // the count is up to three columns long)
    int d = 1;
    for (; d < SAMPLE_MAX && (uint32_t)(d * d) < best; d += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t dd = (uint32_t)((d + u) * (d + u));
            if (j - d - u >= 0)
                best = min(best, __builtin_elementwise_add_sat(dd, gr[j - d - u]));
            if (j + d + u < W)
                best = min(best, __builtin_elementwise_add_sat(dd, gr[j + d + u]));
        }
    }
    return (uint32_t)(d * d) < best ? (uint32_t)ENV_CAP : (uint32_t)d;
}

// edt_rows with g^2 as uint32 in LDS: each strip row holds PAD columns, the
// W values, PAD columns. Without the frame the padding is G2_INF (it cannot
// improve best); with the frame every column outside the window is a feature
// column, g^2 = 0, so the search finds the horizontal distance to the frame
// by itself. A search within PAD columns needs no bounds checks; a saturating
// add keeps g^2 = G2_INF out of the minimum.
//
// Workgroups are dealt to the XCDs round-robin; block b takes strip
// (b % nxcd) * per + b / nxcd, so each XCD takes a contiguous run of strips
// and the strips of one segment read its masks and carries through one L2.
//
// hard_count / hard_list (may be NULL): a strip whose column distances
// average more than ENV_AVG (each counted up to ENV_CAP) and whose sampled
// searches average more than SAMPLE_AVG columns is appended to hard_list and
// left to edt_rows_env (its windowed search would cost about the distance
// per pixel).
template <int STRIP>
__global__ __launch_bounds__(ROWS_BLOCK) void edt_rows32(const uint32_t* __restrict__ mask,
                                                         const int* __restrict__ above,
                                                         const int* __restrict__ below, int H, int W, int frame,
                                                         int nxcd, int per, uint32_t* __restrict__ d2,
                                                         long long ldo, int* __restrict__ hard_count,
                                                         int* __restrict__ hard_list)
{
    extern __shared__ uint32_t g2s[];
    const int WP = W + 2 * PAD;
    const int strip_id = (int)(blockIdx.x % nxcd) * per + (int)(blockIdx.x / nxcd);
    const int r0 = strip_id * STRIP;
    if (r0 >= H)
        return;
    // few columns with a feature (counted by edt_colcarry): edt_rows_env
    // takes every row and this strip only computes its columns
    const bool few_test = hard_list && W > 2 * ENV_FEW;
    // every wave reads the counters (counter lane % FC_PARTS per lane)
    const int part = few_test ? hard_count[fc_index(threadIdx.x & (FC_PARTS - 1))] : 0;
    const int nr = min(STRIP, H - r0);
    const int s = r0 / SEG;
    const uint32_t pad = frame ? 0u : G2_INF;
    for (int t = threadIdx.x; t < nr * 2 * PAD; t += blockDim.x) {
        const int r = t / (2 * PAD), k = t - r * (2 * PAD);
        g2s[r * WP + (k < PAD ? k : W + k)] = pad;
    }
    __shared__ uint32_t s_cost, s_len;
    if (threadIdx.x == 0) {
        s_cost = 0;
        s_len = 0;
    }
    int has = 0;
    uint32_t cost = 0;
    // one column: its g^2 in the strip's rows (into LDS) and its cost
    auto column = [&](int c, uint32_t m, int up0, int dn0) {
        has |= (m != 0) | (up0 >= 0) | (dn0 != NO_ROW_BELOW);
        // nearest feature row above the strip (at or before r0 - 1) and below
        // it (at or after r0 + nr), then running values down and up the strip;
        // "none" is far enough away (2^20 rows) that it never wins a minimum
        // against a real one and is recognised below
        const int b0 = r0 - s * SEG;
        const uint32_t before = b0 ? m & (0xFFFFFFFFu >> (32 - b0)) : 0u;
        const uint32_t after = (b0 + nr < 32) ? m >> (b0 + nr) : 0u;
        constexpr int FAR = 1 << 20;
        int up = before ? s * SEG + 31 - __clz(before) : (up0 >= 0 ? up0 : -FAR);
        int dn = after ? r0 + nr + __ffs(after) - 1 : (dn0 != NO_ROW_BELOW ? dn0 : H + FAR);
        int ups[STRIP];
#pragma unroll
        for (int r = 0; r < STRIP; ++r) {
            if (r < nr && ((m >> (b0 + r)) & 1u))
                up = r0 + r;
            ups[r] = up;
        }
#pragma unroll
        for (int r = STRIP - 1; r >= 0; --r) {
            if (r >= nr)
                continue;
            const int i = r0 + r;
            if ((m >> (b0 + r)) & 1u)
                dn = i;
            int g = min(i - ups[r], dn - i);
            if (frame)
                g = min(g, min(i + 1, H - i));
            // g < 2^16 whenever it is not "none": a 24-bit multiply is exact
            const uint32_t g2 = g >= FAR ? G2_INF : __umul24((uint32_t)g, (uint32_t)g);
            cost += (uint32_t)min(g, ENV_CAP);
            g2s[r * WP + PAD + c] = g2;
        }
    };
#pragma unroll 4
    for (int c = threadIdx.x; c < W; c += blockDim.x)
        column(c, mask[(size_t)s * W + c], above[(size_t)s * W + c], below[(size_t)s * W + c]);
    // few columns with a feature: edt_rows_env takes every row (the test
    // comes after the column loop, where the counters' load has long
    // arrived, so that a strip with work does not wait for it)
    {
        int nfc = part;
#pragma unroll
        for (int o = 1; o < FC_PARTS; o <<= 1)
            nfc += __shfl_xor(nfc, o);
        if (few_test && nfc <= ENV_FEW)
            return;  // uniform
    }
    const int any = __syncthreads_or(has);
    if (!frame && !any) {
        for (int r = 0; r < nr; ++r)
            for (int j = threadIdx.x; j < W; j += blockDim.x)
                d2[(long long)(r0 + r) * ldo + j] = G2_INF;
        return;
    }
    if (hard_list) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            cost += __shfl_xor(cost, o);
        if ((threadIdx.x & 63) == 0)
            atomicAdd(&s_cost, cost);
        __syncthreads();
        if (s_cost > (uint32_t)ENV_AVG * (uint32_t)(nr * W)) {
            // thread t samples row t % nr at a column spread over the row
            const int per = (int)blockDim.x / nr;
            uint32_t len = search_len(g2s, WP, nr, per, W, frame);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                len += __shfl_xor(len, o);
            if ((threadIdx.x & 63) == 0)
                atomicAdd(&s_len, len);
            __syncthreads();
            if (s_len > (uint32_t)SAMPLE_AVG * (uint32_t)(per * nr)) {
                if (threadIdx.x == 0)
                    hard_list[atomicAdd(hard_count, 1)] = strip_id;
                return;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < STRIP; ++r) {
        if (r >= nr)
            break;
        const uint32_t* gr = g2s + r * WP + PAD;
        char* out = reinterpret_cast<char*>(d2 + (long long)(r0 + r) * ldo);
        for (int j = threadIdx.x; j < W; j += blockDim.x)
            *reinterpret_cast<uint32_t*>(out + (uint32_t)j * 4u) = row_min(gr, j, W, frame);
    }
}

// Orders a wave's LDS stores before its lanes' later loads.
__device__ __forceinline__ void env_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The lower envelope of the parabolas (j - x)^2 + g(x)^2 over the columns x
// with a feature is the lower convex hull of the points (x, x^2 + g(x)^2):
// at a pixel j the parabolas' values are j^2 plus a linear function of the
// point, so the lowest is at a hull vertex, and a column whose point lies on
// or above the chord of its two hull neighbours is never strictly lowest.
// Columns are packed with their g as x | g << 16. True when b's point is on
// or above the chord from a's to c's (xa < xb < xc); |values| < 2^34 and
// column gaps < 2^14 keep the products exact in 64 bits.
__device__ __forceinline__ bool env_hidden(uint32_t a, uint32_t b, uint32_t c)
{
    const long long xa = a & 0xFFFFu, xb = b & 0xFFFFu, xc = c & 0xFFFFu;
    const long long ga = a >> 16, gb = b >> 16, gc = c >> 16;
    const long long ya = xa * xa + ga * ga, yb = xb * xb + gb * gb, yc = xc * xc + gc * gc;
    return (yb - ya) * (xc - xb) >= (yc - yb) * (xb - xa);
}

// (j - x)^2 + g^2 for a packed column; H + W <= 65535 keeps it below 2^32
__device__ __forceinline__ uint32_t env_f(uint32_t e, int j)
{
    const int x = (int)(e & 0xFFFFu);
    const uint32_t d = (uint32_t)(j > x ? j - x : x - j);
    const uint32_t g = e >> 16;
    return d * d + g * g;
}

// Per-row state of edt_rows_env shared by its threads: each thread's band of
// the packed columns (then its hull, then its pixels' vertices) at
// E + lane * S, its hull's slice [st, en) of the band, the links of the
// lanes whose slice is not empty, and per merge group (kept at its first
// lane) its first and last lane with a non-empty slice.
struct EnvRow {
    uint32_t* E;
    int S;
    short* st;
    short* en;
    short* prv;
    short* nxt;
    short* gfirst;
    short* glast;
};

// Merges the hulls of the lanes [gl, gl + size) and [gl + size, gl + 2 size)
// (every column of the left group is left of every column of the right
// one): the merged hull is a prefix of the left hull and a suffix of the right
// one, found by removing the left hull's last vertex while it is on or above
// the chord from its predecessor to the right hull's first vertex, and the
// right hull's first vertex while it is on or above the chord from the left
// hull's last vertex to its successor, until neither applies (the common
// lower tangent). A group's first and last vertices are never removed, so a
// group's first and last non-empty lanes stay so. Lanes emptied here are
// unlinked; a link that leaves the group is read as none, so merges of other
// groups that run at the same time never change a decision here.
__device__ void env_merge(const EnvRow& r, int gl, int size)
{
    const int mid = gl + size, ge = gl + 2 * size;
    int Lb = r.glast[gl], Rb = r.gfirst[mid];
    const int first = r.gfirst[gl] >= 0 ? r.gfirst[gl] : r.gfirst[mid];
    const int last = r.glast[mid] >= 0 ? r.glast[mid] : r.glast[gl];
    if (Lb >= 0 && Rb >= 0) {
        for (;;) {
            const uint32_t* eL = r.E + Lb * r.S;
            const uint32_t* eR = r.E + Rb * r.S;
            const uint32_t l1 = eL[r.en[Lb] - 1];
            uint32_t l0 = 0;
            bool has_l0 = false;
            if (r.en[Lb] - 1 > r.st[Lb]) {
                l0 = eL[r.en[Lb] - 2];
                has_l0 = true;
            } else {
                const int m = r.prv[Lb];
                if (m >= gl) {
                    l0 = r.E[m * r.S + r.en[m] - 1];
                    has_l0 = true;
                }
            }
            const uint32_t r0 = eR[r.st[Rb]];
            uint32_t r1 = 0;
            bool has_r1 = false;
            if (r.st[Rb] + 1 < r.en[Rb]) {
                r1 = eR[r.st[Rb] + 1];
                has_r1 = true;
            } else {
                const int m = r.nxt[Rb];
                if (m < ge) {
                    r1 = r.E[m * r.S + r.st[m]];
                    has_r1 = true;
                }
            }
            if (has_l0 && env_hidden(l0, l1, r0)) {
                if (--r.en[Lb] == r.st[Lb]) {
                    // Lb is emptied: a vertex before it (l0) is in the group
                    const int p = r.prv[Lb], q = r.nxt[Lb];
                    r.nxt[p] = (short)q;
                    r.prv[q] = (short)p;
                    Lb = p;
                }
                continue;
            }
            if (has_r1 && env_hidden(l1, r0, r1)) {
                if (++r.st[Rb] == r.en[Rb]) {
                    // Rb is emptied: a vertex after it (r1) is in the group
                    const int p = r.prv[Rb], q = r.nxt[Rb];
                    if (p >= 0)
                        r.nxt[p] = (short)q;
                    r.prv[q] = (short)p;
                    Rb = q;
                }
                continue;
            }
            break;
        }
    }
    r.gfirst[gl] = (short)first;
    r.glast[gl] = (short)last;
}

// Phase 2 of the rows of the strips that edt_rows32 listed: Alg. 2's lower
// envelope, built in parallel, one row per workgroup of ENV_NT threads,
// whatever the row's distances:
//   g of the row from the masks and carries, packed with the column into the
//   threads' bands of B columns (B the least power of two with B ENV_NT >= W;
//   a band at a stride of S = B | 1 entries, so neighbouring bands start in
//   different LDS banks). The frame is left out of g: the distance to the
//   outside of the window is (i + 1)^2, (H - i)^2, (j + 1)^2 or (W - j)^2,
//   and the minimum over the features and the outside is the minimum of the
//   transform without the frame and those four, taken at the end; so a
//   sparse row keeps few columns with a feature whether or not the frame
//   counts;
//   each thread builds the lower hull of its band with a stack, in place (Alg.
//   2's first scan, on its band);
//   the hulls are merged pairwise in log2(ENV_NT) rounds (one thread per
//   pair);
//   the hull's vertices are gathered in column order (vertex t at t + t / B);
//   each thread finds the vertex lowest at the first pixel of its band by
//   bisection (along the hull the values at a fixed pixel fall, then rise)
//   and walks forward through its band (Alg. 2's second scan), noting each
//   pixel's vertex in its band;
//   the row is written from those, coalesced.
__global__ __launch_bounds__(ENV_NT) void edt_rows_env(const uint32_t* __restrict__ mask,
                                                       const int* __restrict__ above,
                                                       const int* __restrict__ below, int H, int W, int frame,
                                                       int strip, const int* __restrict__ hard_count,
                                                       const int* __restrict__ hard_list,
                                                       const uint16_t* __restrict__ fcb, uint32_t* __restrict__ d2,
                                                       long long ldo)
{
    extern __shared__ uint32_t env_sm[];
    // (short: with 4 bytes each, four workgroups would not fit a CU at W = 4096)
    __shared__ short st[ENV_NT], en[ENV_NT], prv[ENV_NT], nxt[ENV_NT], gfirst[ENV_NT], glast[ENV_NT];
    __shared__ int s_wave[2][ENV_NT / 64];
    // the image's columns with a feature in increasing order when there are
    // at most ENV_FEW, and their g^2 in the current row
    __shared__ int fc_k[ENV_FEW];
    __shared__ uint32_t fc_g2[ENV_FEW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lb = 31 - __clz((unsigned)((W + ENV_NT - 1) / ENV_NT * 2 - 1));  // B = 2^lb
    const int B = 1 << lb;
    const int S = B | 1;
    const EnvRow r{env_sm, S, st, en, prv, nxt, gfirst, glast};
    uint32_t* band = env_sm + tid * S;
    uint32_t* hull = env_sm + ENV_NT * S;
    const int c0 = min(W, tid * B), nb = min(W, c0 + B) - c0;
    // few columns with a feature (W > 2 ENV_FEW): every row, which
    // edt_rows32 left unread; else the rows of the listed strips
    const int nfc = feature_columns(hard_count);
    const bool all_rows = W > 2 * ENV_FEW && nfc <= ENV_FEW;
    const int nrows = all_rows ? H : hard_count[0] * strip;
    if (nrows == 0)
        return;
    // the columns with a feature (edt_colcarry's bits and count), in
    // increasing order when there are few: thread t takes Q consecutive bit
    // words and places its columns after those of the threads before it
    if (nfc <= ENV_FEW) {
        const int nwd = (W + 15) / 16, Q = (nwd + ENV_NT - 1) / ENV_NT;
        int cnt = 0;
        for (int q = 0; q < Q; ++q) {
            const int w = tid * Q + q;
            cnt += w < nwd ? __popc((uint32_t)fcb[w]) : 0;
        }
        int pre = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(pre, o);
            if (lane >= o)
                pre += v;
        }
        if (lane == 63)
            s_wave[0][wave] = pre;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < ENV_NT / 64; ++w)
            pre += w < wave ? s_wave[0][w] : 0;
        pre -= cnt;
        for (int q = 0; q < Q && cnt; ++q) {
            const int w = tid * Q + q;
            uint32_t bits = w < nwd ? (uint32_t)fcb[w] : 0u;
            while (bits) {
                const int l = __ffs(bits) - 1;
                bits &= bits - 1u;
                fc_k[pre++] = w * 16 + l;
            }
        }
        __syncthreads();
    }
    // few: each thread's run of B consecutive pixels (B: the band width,
    // B * ENV_NT >= W), staged at j + j / B so that the threads' runs start
    // in different banks; (j - k)^2 + g^2 < 2^32 with 24-bit multiplies
    // (|j - k| and g below 2^16)
    const int j0 = min(W, tid * B), j1 = min(W, j0 + B);
    auto few_f = [&](int q, int j) {
        const int k = fc_k[q];
        const uint32_t d = (uint32_t)(j > k ? j - k : k - j);
        return __umul24(d, d) + fc_g2[q];
    };
    for (int b = blockIdx.x; b < nrows; b += gridDim.x) {
        const int i = all_rows ? b : hard_list[b / strip] * strip + b % strip;
        if (i >= H)
            continue;  // uniform: a strip's rows past the image
        const int s = i / SEG;
        const int bi = i - s * SEG;
        const size_t base = (size_t)s * W;
        if (nfc <= ENV_FEW) {
            if (tid < nfc) {
                const int c = fc_k[tid];
                const uint32_t m = mask[base + c];
                const uint32_t lo = m & (0xFFFFFFFFu >> (31 - bi));
                const uint32_t hi = m >> bi;
                const int up = lo ? s * SEG + 31 - __clz(lo) : above[base + c];
                const int dn = hi ? i + __ffs(hi) - 1 : below[base + c];
                int v = NO_ROW_BELOW;
                if (up >= 0)
                    v = i - up;
                if (dn != NO_ROW_BELOW)
                    v = min(v, dn - i);
                fc_g2[tid] = __umul24((uint32_t)v, (uint32_t)v);  // finite: the column holds a feature
            }
            __syncthreads();
            uint32_t* out = d2 + (long long)i * ldo;
            const uint32_t fv = frame ? (uint32_t)min(i + 1, H - i) * (uint32_t)min(i + 1, H - i) : G2_INF;
            if (j0 < j1) {
                // the first column (in increasing order) that is lowest at
                // the run's first and last pixels: lowest columns only move
                // right as j grows (two parabolas of equal width cross
                // once), so at every pixel of the run a lowest column lies
                // between them
                int qa = 0, qb = 0;
                uint32_t va = G2_INF, vb = G2_INF;
                for (int q = 0; q < nfc; ++q) {
                    const uint32_t fa = few_f(q, j0), fb = few_f(q, j1 - 1);
                    if (fa < va) {
                        va = fa;
                        qa = q;
                    }
                    if (fb < vb) {
                        vb = fb;
                        qb = q;
                    }
                }
                for (int j = j0; j < j1; ++j) {
                    uint32_t v = G2_INF;
                    for (int q = qa; q <= qb && q < nfc; ++q)
                        v = min(v, few_f(q, j));
                    env_sm[j + (j >> lb)] = v;  // staged, then written coalesced
                }
            }
            __syncthreads();
            // the row is written from a rotated start (whole 64-column
            // chunks), so that the workgroups writing rows at the same time
            // are not all at the same offsets of their rows
            const int rot = (int)(((unsigned)i * 37u) % (unsigned)((W + 63) / 64)) * 64;
            for (int jj = tid; jj < W; jj += ENV_NT) {
                const int j = jj + rot < W ? jj + rot : jj + rot - W;
                uint32_t v = env_sm[j + (j >> lb)];
                if (frame) {
                    const uint32_t e = (uint32_t)min(j + 1, W - j);
                    v = min(v, min(fv, __umul24(e, e)));
                }
                out[j] = v;
            }
            __syncthreads();  // the next row rewrites the columns' values and the staging
            continue;
        }
#pragma unroll 8
        for (int c = tid; c < W; c += ENV_NT) {
            const uint32_t m = mask[base + c];
            const int up0 = above[base + c];
            const int dn0 = below[base + c];
            const uint32_t lo = m & (0xFFFFFFFFu >> (31 - bi));  // rows <= i in the segment
            const uint32_t hi = m >> bi;                         // rows >= i
            const int up = lo ? s * SEG + 31 - __clz(lo) : up0;
            const int dn = hi ? i + __ffs(hi) - 1 : dn0;
            int v = NO_ROW_BELOW;
            if (up >= 0)
                v = i - up;
            if (dn != NO_ROW_BELOW)
                v = min(v, dn - i);
            const uint32_t g = v == NO_ROW_BELOW ? G_INF : (uint32_t)v;
            env_sm[(c >> lb) * S + (c & (B - 1))] = (uint32_t)c | g << 16;
        }
        __syncthreads();
        // the band's hull, a stack over the band's own entries
        int k = 0;
        for (int t = 0; t < nb; ++t) {
            const uint32_t e = band[t];
            if ((e >> 16) == G_INF)
                continue;
            while (k >= 2 && env_hidden(band[k - 2], band[k - 1], e))
                --k;
            band[k++] = e;
        }
        st[tid] = 0;
        en[tid] = (short)k;
        // links of the non-empty lanes: the nearest non-empty lane before and
        // after each lane (scans over the workgroup), -1 and ENV_NT for none
        {
            int lo_v = k ? tid : -1, hi_v = k ? tid : ENV_NT;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int a = __shfl_up(lo_v, o), c = __shfl_down(hi_v, o);
                if (lane >= o)
                    lo_v = max(lo_v, a);
                if (lane + o < 64)
                    hi_v = min(hi_v, c);
            }
            if (lane == 63)
                s_wave[0][wave] = lo_v;
            if (lane == 0)
                s_wave[1][wave] = hi_v;
            __syncthreads();
            int carry_lo = -1, carry_hi = ENV_NT;
#pragma unroll
            for (int w = 0; w < ENV_NT / 64; ++w) {
                if (w < wave)
                    carry_lo = max(carry_lo, s_wave[0][w]);
                if (w > wave)
                    carry_hi = min(carry_hi, s_wave[1][w]);
            }
            // exclusive: the lanes strictly before and after this one
            int pe = __shfl_up(lo_v, 1), ne = __shfl_down(hi_v, 1);
            pe = lane == 0 ? carry_lo : max(pe, carry_lo);
            ne = lane == 63 ? carry_hi : min(ne, carry_hi);
            prv[tid] = (short)pe;
            nxt[tid] = (short)ne;
            gfirst[tid] = (short)(k ? tid : -1);
            glast[tid] = (short)(k ? tid : -1);
        }
        __syncthreads();
        for (int size = 1; size < ENV_NT; size <<= 1) {
            if ((tid & (2 * size - 1)) == 0)
                env_merge(r, tid, size);
            __syncthreads();
        }
        // gather the hull in column order (an exclusive scan of the slices)
        const int cnt = en[tid] - st[tid];
        int pre = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(pre, o);
            if (lane >= o)
                pre += v;
        }
        if (lane == 63)
            s_wave[0][wave] = pre;
        __syncthreads();
        int n = 0;
#pragma unroll
        for (int w = 0; w < ENV_NT / 64; ++w) {
            pre += w < wave ? s_wave[0][w] : 0;
            n += s_wave[0][w];
        }
        pre -= cnt;
        for (int t = 0; t < cnt; ++t) {
            const int h = pre + t;
            hull[h + (h >> lb)] = band[st[tid] + t];
        }
        __syncthreads();  // the bands are free once the hull is gathered
        uint32_t* out = d2 + (long long)i * ldo;
        // the frame's rows above and below (none: G2_INF)
        const uint32_t fv = frame ? (uint32_t)min(i + 1, H - i) * (uint32_t)min(i + 1, H - i) : G2_INF;
        if (n == 0) {
            // no feature in any column: only the frame
            for (int j = tid; j < W; j += ENV_NT) {
                const uint32_t e = (uint32_t)min(j + 1, W - j);
                out[j] = frame ? min(fv, e * e) : G2_INF;
            }
            continue;
        }
        if (nb > 0) {
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int m1 = mid + 1;
                if (env_f(hull[m1 + (m1 >> lb)], c0) <= env_f(hull[mid + (mid >> lb)], c0))
                    lo = m1;
                else
                    hi = mid;
            }
            int t = lo;
            uint32_t cur = hull[t + (t >> lb)];
            for (int j = 0; j < nb; ++j) {
                while (t + 1 < n) {
                    const int t1 = t + 1;
                    const uint32_t nx = hull[t1 + (t1 >> lb)];
                    if (env_f(nx, c0 + j) > env_f(cur, c0 + j))
                        break;
                    t = t1;
                    cur = nx;
                }
                band[j] = cur;
            }
        }
        __syncthreads();
        for (int j = tid; j < W; j += ENV_NT) {
            uint32_t v = env_f(env_sm[(j >> lb) * S + (j & (B - 1))], j);
            if (frame) {
                const uint32_t e = (uint32_t)min(j + 1, W - j);
                v = min(v, min(fv, e * e));
            }
            out[j] = v;
        }
        __syncthreads();  // the next row rewrites the bands and the hull
    }
}

}  // namespace

namespace hasf_detail {

size_t edt_scratch_bytes(int H, int W)
{
    const size_t nseg = (size_t)(H + SEG - 1) / SEG;
    // masks, carries above and below; the count and list of strips for edt_rows_env
    // and the feature columns' bits (one uint16 per 16 columns)
    return nseg * W * (sizeof(uint32_t) + 2 * sizeof(int)) + 3 * 256 + CTL_INTS * sizeof(int) +
           ((size_t)H * sizeof(int) + 255) / 256 * 256 +
           ((size_t)(W + 15) / 16 * sizeof(uint16_t) + 255) / 256 * 256;
}

// scratch: device memory of edt_scratch_bytes(H, W)
// invert != 0: the features are the zero bytes of F instead of the nonzero ones
hipError_t launch_edt(const uint8_t* F, int H, int W, long long ld, int frame, int invert, uint32_t* d2,
                      long long ldo, void* scratch, size_t lds_max, int nxcd, hipStream_t stream)
{
    nxcd = std::max(1, nxcd);
    const int nseg = (H + SEG - 1) / SEG;
    char* p = (char*)scratch;
    uint32_t* mask = (uint32_t*)p;
    p += ((size_t)nseg * W * sizeof(uint32_t) + 255) / 256 * 256;
    int* above = (int*)p;
    p += ((size_t)nseg * W * sizeof(int) + 255) / 256 * 256;
    int* below = (int*)p;
    p += ((size_t)nseg * W * sizeof(int) + 255) / 256 * 256;
    int* hard_count = (int*)p;
    p += CTL_INTS * sizeof(int);
    int* hard_list = (int*)p;  // at most one entry per row
    p += ((size_t)H * sizeof(int) + 255) / 256 * 256;
    uint16_t* fcb = (uint16_t*)p;  // counted by the counters after hard_count[0]
    // rows up to ENV_W_MAX wide that edt_rows32 takes get the envelope for far strips
    const bool env = W <= ENV_W_MAX;

    const int vec4 = ((((uintptr_t)F) | (uintptr_t)ld) & 3) == 0;
    hipLaunchKernelGGL(edt_colmask, dim3((W + 1023) / 1024, nseg), dim3(256), 0, stream, F, ld, H, W, invert, vec4,
                       mask, env ? hard_count : nullptr);
    hipLaunchKernelGGL(edt_colcarry, dim3((W + CARRY_COLS - 1) / CARRY_COLS), dim3(CARRY_COLS * CARRY_GROUPS), 0,
                       stream, mask, nseg, W, above, below, env ? fcb : nullptr, env ? hard_count : nullptr);
    // strip height: a divisor of 32 (a strip lies in one segment), as LDS
    // allows (1 KiB is left for the kernels' static LDS): up to 4 rows of
    // padded uint32 g^2 in half the LDS (two workgroups per CU), else in all
    // of it, else up to 8 rows of uint16 g
    const size_t lds_dyn = lds_max - 1024;
    const int block = std::min(512, std::max(256, (W + 63) / 64 * 64));
    static std::atomic<uint64_t> attr_rows{0}, attr_r4{0}, attr_r2{0}, attr_r1{0};
    hipError_t e = allow_dyn_lds((const void*)edt_rows, (int)lds_dyn, attr_rows);
    if (e == hipSuccess)
        e = allow_dyn_lds((const void*)edt_rows32<4>, (int)lds_dyn, attr_r4);
    if (e == hipSuccess)
        e = allow_dyn_lds((const void*)edt_rows32<2>, (int)lds_dyn, attr_r2);
    if (e == hipSuccess)
        e = allow_dyn_lds((const void*)edt_rows32<1>, (int)lds_dyn, attr_r1);
    if (e != hipSuccess)
        return e;
    const size_t row32 = (size_t)(W + 2 * PAD) * 4;
    if (row32 <= lds_dyn) {
        // two rows per strip and 512 threads: four workgroups share a CU, so
        // one's global loads overlap the others' searches (measured best at
        // 4096^2 among 1, 2, 4 rows and 256 to 1024 threads)
        int strip = 2;
        while (strip > 1 && strip * row32 > lds_dyn / 4)
            strip >>= 1;
        const int nstrips = (H + strip - 1) / strip;
        const int per = (nstrips + nxcd - 1) / nxcd;
        const dim3 grid(per * nxcd);
        int* hc = env ? hard_count : nullptr;
        int* hl = env ? hard_list : nullptr;
        if (strip == 4)
            hipLaunchKernelGGL(edt_rows32<4>, grid, dim3(block), 4 * row32, stream, mask, above, below, H, W, frame,
                               nxcd, per, d2, ldo, hc, hl);
        else if (strip == 2)
            hipLaunchKernelGGL(edt_rows32<2>, grid, dim3(block), 2 * row32, stream, mask, above, below, H, W, frame,
                               nxcd, per, d2, ldo, hc, hl);
        else
            hipLaunchKernelGGL(edt_rows32<1>, grid, dim3(block), row32, stream, mask, above, below, H, W, frame,
                               nxcd, per, d2, ldo, hc, hl);
        if (env) {
            // the listed strips' rows, a row per workgroup (nothing when
            // nothing was listed: each workgroup reads the count and ends);
            // LDS: the bands (ENV_NT * (B | 1) entries) and the hull (up to
            // W + W / B entries), uint32 each
            int B = 1;
            while (B * ENV_NT < W)
                B <<= 1;
            const size_t row_lds = ((size_t)ENV_NT * (B | 1) + W + W / B + 2) * 4;
            static std::atomic<uint64_t> attr_env{0};
            // (its static LDS, the lanes' slices and links, is under 4 KiB)
            const hipError_t ee = allow_dyn_lds((const void*)edt_rows_env, (int)(lds_dyn - 4096), attr_env);
            if (ee != hipSuccess)
                return ee;
            const int rows = nstrips * strip;
            // four workgroups per CU (the LDS allows four at W = 4096); few
            // workgroups also keep the launch cheap when nothing was listed
            const int egrid = std::max(1, std::min(rows, 1024));
            hipLaunchKernelGGL(edt_rows_env, dim3(egrid), dim3(ENV_NT), row_lds, stream, mask, above, below, H, W,
                               frame, strip, hard_count, hard_list, fcb, d2, ldo);
        }
        return hipGetLastError();
    }
    int strip = 8;
    while (strip > 1 && (size_t)strip * W * 2 > lds_dyn)
        strip >>= 1;
    hipLaunchKernelGGL(edt_rows, dim3((H + strip - 1) / strip), dim3(block), (size_t)strip * W * 2, stream, mask,
                       above, below, H, W, frame, strip, d2, ldo);
    return hipGetLastError();
}

}  // namespace hasf_detail

// ---------------------------------------------------------------------------
// Scratch of the allocation-free EDT entry point: the segment masks and
// carries live in this file-scope array instead of the context's growable
// scratch. Host code never passes the array's name to a kernel (on the host
// it is a stand-in, not a device address): noalloc_init takes each device's
// address of its own copy once, with that device current, and every launch
// uses that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HASF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES];
}  // namespace

namespace hasf_detail {

hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device])
        return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_noalloc_ptr[device] = p;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

}  // namespace hasf_detail
