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
// carries; the per-column g never leaves LDS.
#include "hasf_common.h"

namespace {

constexpr int SEG = 32;
constexpr uint16_t G_INF = 0xFFFF;
constexpr int ROWS_BLOCK = 256;

__global__ __launch_bounds__(256) void edt_colmask(const uint8_t* __restrict__ F, long long ld, int H, int W,
                                                   int invert, uint32_t* __restrict__ mask, int* __restrict__ any)
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
    if (m)
        *any = 1;  // benign race: every writer stores 1
}

// above[s*W+c] = nearest feature row < s*SEG (or -1); below = nearest >= (s+1)*SEG (or INT_MAX)
__global__ __launch_bounds__(256) void edt_colcarry(const uint32_t* __restrict__ mask, int nseg, int W,
                                                    int* __restrict__ above, int* __restrict__ below)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= W)
        return;
    int last = -1;
    for (int s = 0; s < nseg; ++s) {
        above[(size_t)s * W + c] = last;
        const uint32_t m = mask[(size_t)s * W + c];
        if (m)
            last = s * SEG + 31 - __clz(m);
    }
    int first = 0x7FFFFFFF;
    for (int s = nseg - 1; s >= 0; --s) {
        below[(size_t)s * W + c] = first;
        const uint32_t m = mask[(size_t)s * W + c];
        if (m)
            first = s * SEG + __ffs(m) - 1;
    }
}

__global__ __launch_bounds__(ROWS_BLOCK) void edt_rows(const uint32_t* __restrict__ mask,
                                                       const int* __restrict__ above,
                                                       const int* __restrict__ below, int H, int W,
                                                       int frame, int strip, const int* __restrict__ any,
                                                       uint32_t* __restrict__ d2, long long ldo)
{
    extern __shared__ uint16_t gs[];
    const int r0 = blockIdx.x * strip;
    const int nr = min(strip, H - r0);
    if (!frame && *any == 0) {
        for (int r = 0; r < nr; ++r)
            for (int j = threadIdx.x; j < W; j += blockDim.x)
                d2[(long long)(r0 + r) * ldo + j] = 0xFFFFFFFFu;
        return;
    }
    // phase 1: g of the strip into LDS
    for (int c = threadIdx.x; c < W; c += blockDim.x) {
        for (int r = 0; r < nr; ++r) {
            const int i = r0 + r;
            const int s = i / SEG;
            const int b = i - s * SEG;
            const uint32_t m = mask[(size_t)s * W + c];
            const uint32_t lo = m & (0xFFFFFFFFu >> (31 - b));  // rows <= i in the segment
            const uint32_t hi = m >> b;                         // rows >= i
            const int up = lo ? s * SEG + 31 - __clz(lo) : above[(size_t)s * W + c];
            const int dn = hi ? i + __ffs(hi) - 1 : below[(size_t)s * W + c];
            int g = 0x7FFFFFFF;
            if (up >= 0)
                g = i - up;
            if (dn != 0x7FFFFFFF)
                g = min(g, dn - i);
            if (frame)
                g = min(g, min(i + 1, H - i));
            gs[r * W + c] = g == 0x7FFFFFFF ? G_INF : (uint16_t)g;
        }
    }
    __syncthreads();
    // phase 2: per pixel, exact minimum over columns by increasing |j - k|
    for (int r = 0; r < nr; ++r) {
        const uint16_t* gr = gs + r * W;
        for (int j = threadIdx.x; j < W; j += blockDim.x) {
            const uint32_t g0 = gr[j];
            uint32_t best = g0 == G_INF ? 0xFFFFFFFFu : g0 * g0;
            if (frame) {
                const uint32_t e = (uint32_t)min(j + 1, W - j);
                best = min(best, e * e);
            }
            for (int d = 1;; ++d) {
                const uint32_t dd = (uint32_t)d * (uint32_t)d;
                if (dd >= best)
                    break;
                const bool lft = j - d >= 0, rgt = j + d < W;
                if (!lft && !rgt)
                    break;
                if (lft) {
                    const uint32_t g = gr[j - d];
                    if (g != G_INF)
                        best = min(best, dd + g * g);
                }
                if (rgt) {
                    const uint32_t g = gr[j + d];
                    if (g != G_INF)
                        best = min(best, dd + g * g);
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
    return 256 + nseg * W * (sizeof(uint32_t) + 2 * sizeof(int)) + 3 * 256;
}

// scratch: device memory of edt_scratch_bytes(H, W)
// invert != 0: the features are the zero bytes of F instead of the nonzero ones
hipError_t launch_edt(const uint8_t* F, int H, int W, long long ld, int frame, int invert, uint32_t* d2,
                      long long ldo, void* scratch, size_t lds_max, hipStream_t stream)
{
    const int nseg = (H + SEG - 1) / SEG;
    char* p = (char*)scratch;
    int* any = (int*)p;
    p += 256;
    uint32_t* mask = (uint32_t*)p;
    p += ((size_t)nseg * W * sizeof(uint32_t) + 255) / 256 * 256;
    int* above = (int*)p;
    p += ((size_t)nseg * W * sizeof(int) + 255) / 256 * 256;
    int* below = (int*)p;

    hipError_t e = hipMemsetAsync(any, 0, sizeof(int), stream);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(edt_colmask, dim3((W + 255) / 256, nseg), dim3(256), 0, stream, F, ld, H, W, invert, mask, any);
    hipLaunchKernelGGL(edt_colcarry, dim3((W + 255) / 256), dim3(256), 0, stream, mask, nseg, W, above, below);
    // strip height: as many rows of uint16 g as LDS allows, at most 16
    int strip = (int)min((size_t)16, lds_max / (2 * (size_t)W));
    if (strip < 1)
        strip = 1;
    const size_t lds = (size_t)strip * W * 2;
    static bool attr = false;
    if (!attr) {
        e = hipFuncSetAttribute((const void*)edt_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_max);
        if (e != hipSuccess)
            return e;
        attr = true;
    }
    hipLaunchKernelGGL(edt_rows, dim3((H + strip - 1) / strip), dim3(ROWS_BLOCK), lds, stream, mask, above,
                       below, H, W, frame, strip, any, d2, ldo);
    return hipGetLastError();
}

}  // namespace hasf_detail
