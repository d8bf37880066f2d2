// Exact squared Euclidean distance transform on gfx950 (Sec. 4.1).
//
// The transform is separable: d2(i, j) = min_k (j - k)^2 + g(i, k)^2 where
// g(i, k) is the distance from row i to the nearest feature of column k
// (phase 1, columns; phase 2, rows). The paper's CPU version deals whole
// columns and whole rows to threads; a column scan is sequential in rows, so
// here phase 1 is split into 32-row segments that are independent:
//
//   edt_colmask   one thread per (column, 32-row segment): the segment's
//                 features as a 32-bit mask (reads the input once).
//   edt_colcarry  one thread per column: for every segment, the nearest
//                 feature row above the segment and below it (a prefix-max /
//                 suffix-min over the segment masks).
//   edt_rows      one workgroup per strip of rows: g of the strip from the
//                 masks and carries (O(1) per pixel with clz/ctz), kept in
//                 LDS, then phase 2 per pixel as an exact windowed minimum:
//                 starting from g(i, j)^2, columns j -+ 1, j -+ 2, ... are
//                 visited until d^2 reaches the best value found, beyond which
//                 no column can improve it. The result is written once.
//
// HBM traffic: 1 B/px read + 4 B/px written, plus 3/8 B/px of masks and
// carries; the per-column g never leaves LDS. With no feature at all (and no
// frame) every column is empty, which the strip kernel sees by itself.
#include "hasf_common.h"

namespace {

constexpr int SEG = 32;
constexpr uint16_t G_INF = 0xFFFF;
constexpr int ROWS_BLOCK = 1024;
constexpr int NO_ROW_BELOW = 0x7FFFFFFF;

// one thread per (column, 32-row segment): the segment's features as a mask
__global__ __launch_bounds__(256) void edt_colmask(const uint8_t* __restrict__ F, long long ld, int H, int W,
                                                   int invert, uint32_t* __restrict__ mask)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (c >= W)
        return;
    const int r0 = s * SEG;
    const int n = min(SEG, H - r0);
    const uint8_t* p = F + (long long)r0 * ld + c;
    uint32_t m = 0;
#pragma unroll 8
    for (int b = 0; b < n; ++b)
        m |= (uint32_t)((p[(long long)b * ld] != 0) != (invert != 0)) << b;
    mask[(size_t)s * W + c] = m;
}

// Per column and segment: the nearest feature row above the segment
// (above, -1 if none) and below it (below, NO_ROW_BELOW if none). A block
// covers 64 columns; the 4 threads of a column split its segments into 4
// consecutive groups, scan them, and combine through LDS.
__global__ __launch_bounds__(256) void edt_colcarry(const uint32_t* __restrict__ mask, int nseg, int W,
                                                    int* __restrict__ above, int* __restrict__ below)
{
    __shared__ int glast[4][64], gfirst[4][64];
    const int lc = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lc;
    const int G = (nseg + 3) >> 2;
    const int s0 = grp * G, s1 = min(nseg, s0 + G);
    int last = -1, first = NO_ROW_BELOW;
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
    if (c >= W)
        return;
    int up = -1, dn = NO_ROW_BELOW;
    for (int k = 0; k < grp; ++k)
        up = max(up, glast[k][lc]);
    for (int k = 3; k > grp; --k)
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

}  // namespace

namespace hasf_detail {

size_t edt_scratch_bytes(int H, int W)
{
    const size_t nseg = (size_t)(H + SEG - 1) / SEG;
    return nseg * W * (sizeof(uint32_t) + 2 * sizeof(int)) + 3 * 256;
}

// scratch: device memory of edt_scratch_bytes(H, W)
// invert != 0: the features are the zero bytes of F instead of the nonzero ones
hipError_t launch_edt(const uint8_t* F, int H, int W, long long ld, int frame, int invert, uint32_t* d2,
                      long long ldo, void* scratch, size_t lds_max, hipStream_t stream)
{
    const int nseg = (H + SEG - 1) / SEG;
    char* p = (char*)scratch;
    uint32_t* mask = (uint32_t*)p;
    p += ((size_t)nseg * W * sizeof(uint32_t) + 255) / 256 * 256;
    int* above = (int*)p;
    p += ((size_t)nseg * W * sizeof(int) + 255) / 256 * 256;
    int* below = (int*)p;

    hipLaunchKernelGGL(edt_colmask, dim3((W + 255) / 256, nseg), dim3(256), 0, stream, F, ld, H, W, invert, mask);
    hipLaunchKernelGGL(edt_colcarry, dim3((W + 63) / 64), dim3(256), 0, stream, mask, nseg, W, above, below);
    // strip height: a divisor of 32, at most 8 rows, as LDS allows (1 KiB is
    // left for the kernel's static LDS)
    const size_t lds_dyn = lds_max - 1024;
    int strip = 8;
    while (strip > 1 && (size_t)strip * W * 2 > lds_dyn)
        strip >>= 1;
    const size_t lds = (size_t)strip * W * 2;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)edt_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_dyn);
        if (e != hipSuccess)
            return e;
        attr = true;
    }
    hipLaunchKernelGGL(edt_rows, dim3((H + strip - 1) / strip), dim3(ROWS_BLOCK), lds, stream, mask, above,
                       below, H, W, frame, strip, d2, ldo);
    return hipGetLastError();
}

}  // namespace hasf_detail
