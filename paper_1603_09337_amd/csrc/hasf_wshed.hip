// The topological watershed's lowering (grey-level W-thinning) on 2D
// grey-level images. The paper places the topological watershed in the same
// class of topology-based operators as its filter (Sec. 3.1); the operator
// here is the classical grey-level one on the (8,4) pair of Sec. 2:
//   - lower sections {p : F(p) < k} are 4-connected; the plane outside the
//     window never belongs to one;
//   - a pixel p is W-destructible when it has a lower neighbour and the
//     lower pixels of its 8-neighbourhood that are 4-adjacent to p lie in one
//     4-component of the neighbourhood's lower pixels (T-bar = 1);
//   - a W-destructible p is lowered to the largest level among its lower
//     neighbours (its neighbourhood's lower pixels are then the same for every
//     level in between, so it stays W-destructible all the way down);
//   - rounds of four passes over the 2x2 parity subfields of (row, column),
//     until a round lowers nothing (two pixels of one subfield are never
//     8-adjacent, so a pass is a data-parallel map).
// Lowering joins exactly one lower component and never merges two, so every
// lower section keeps its components (no merge, no new minimum).
//
// One workgroup lowers one image at a time (a persistent queue over the
// batch), in place in the caller's buffer. Only a pixel lowered in the
// previous passes, or next to one, can become W-destructible, so a pass tests
// the pixels of the flagged 64-column words of its subfield only.
#include "hasf_common.h"

namespace {

constexpr int WS_NT = 1024;
constexpr int WS_FLAG_BYTES_MAX = 96 * 1024;  // LDS flags: 4 bytes per row and 64-column word

// T-bar = 1 for a neighbourhood code (bit k set: neighbour k is not lower;
// neighbours in the order E NE N NW W SW S SE, consecutive ones 4-adjacent):
// the lower positions form circular runs, and the runs that hold a 4-neighbour
// (an even position) are the 4-components adjacent to the centre.
struct WsTables {
    uint32_t one[8];  // bit m of the 256-bit table
};

constexpr WsTables make_ws_tables()
{
    WsTables t{};
    for (int m = 0; m < 256; ++m) {
        const int low = ~m & 0xFF;
        int comps = 0;
        if (low == 0xFF) {
            comps = 1;
        } else if (low != 0) {
            // start after a non-lower position, walk the ring once
            int start = 0;
            while ((low >> start) & 1)
                ++start;
            bool in_run = false, has4 = false;
            for (int s = 1; s <= 8; ++s) {
                const int k = (start + s) & 7;
                if ((low >> k) & 1) {
                    in_run = true;
                    has4 |= (k & 1) == 0;
                } else if (in_run) {
                    comps += has4 ? 1 : 0;
                    in_run = false;
                    has4 = false;
                }
            }
        }
        if (comps == 1)
            t.one[m >> 5] |= 1u << (m & 31);
    }
    return t;
}

__constant__ WsTables WT = make_ws_tables();

__device__ __forceinline__ bool ws_tbar1(unsigned m)
{
    return (WT.one[m >> 5] >> (m & 31)) & 1u;
}

// Tests pixel (i, j); lowers it when W-destructible. Returns whether it did.
__device__ __forceinline__ bool ws_pixel(uint8_t* F, long long ld, int H, int W, int i, int j)
{
    uint8_t* p = F + (long long)i * ld + j;
    const int v = *p;
    const bool up = i > 0, dn = i < H - 1, lf = j > 0, rt = j < W - 1;
    // E NE N NW W SW S SE; outside: not lower
    const int n0 = rt ? p[1] : 256;
    const int n1 = (up && rt) ? p[-ld + 1] : 256;
    const int n2 = up ? p[-ld] : 256;
    const int n3 = (up && lf) ? p[-ld - 1] : 256;
    const int n4 = lf ? p[-1] : 256;
    const int n5 = (dn && lf) ? p[ld - 1] : 256;
    const int n6 = dn ? p[ld] : 256;
    const int n7 = (dn && rt) ? p[ld + 1] : 256;
    const int nb[8] = {n0, n1, n2, n3, n4, n5, n6, n7};
    unsigned m = 0;
    int delta = -1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (nb[k] >= v)
            m |= 1u << k;
        else
            delta = nb[k] > delta ? nb[k] : delta;
    }
    if (delta < 0 || !ws_tbar1(m))
        return false;
    *p = (uint8_t)delta;
    return true;
}

}  // namespace

// Each workgroup claims images in queue order until none is left. Flags (LDS,
// when the image's fit, else every word is tested): one byte per row, 64-column
// word and column parity, for the coming passes (cur) and set by this pass's
// lowerings (nxt); a pass tests the pixels of its subfield whose word is
// flagged for their column parity, then its own flags are replaced by this
// pass's and the others' gain them.
__global__ __launch_bounds__(WS_NT) void hasf_wshed_kernel(const GreyDesc* __restrict__ desc, int n,
                                                           int* __restrict__ next)
{
    extern __shared__ uint8_t ws_flags[];  // cur[2][rows x words], nxt[2][rows x words]
    __shared__ int s_img, s_flag;
    for (;;) {
        if (threadIdx.x == 0)
            s_img = atomicAdd(next, 1);
        __syncthreads();
        const int img = s_img;
        __syncthreads();
        if (img >= n)
            break;
        const GreyDesc& d = desc[img];
        uint8_t* F = d.F;
        const int H = d.H, W = d.W;
        const long long ld = d.ld;
        const int WW = (W + 63) >> 6;
        const bool flags = d.flags != 0;
        const int nf = flags ? H * WW : 0;
        uint8_t* cur = ws_flags;       // [2][nf]
        uint8_t* nxt = ws_flags + 2 * nf;
        for (int q = threadIdx.x; q < 2 * nf; q += WS_NT) {
            cur[q] = 1;  // every word is tested at first
            nxt[q] = 0;
        }
        __syncthreads();
        for (;;) {
            if (threadIdx.x == 0)
                s_flag = 0;
            __syncthreads();
            for (int s = 0; s < 4; ++s) {
                const int si = s >> 1, sj = s & 1;
                const int rows = (H - si + 1) >> 1;
                const int cols = (W - sj + 1) >> 1;
                bool changed = false;
                for (int t = threadIdx.x; t < rows * cols; t += WS_NT) {
                    const int ri = t / cols;
                    const int i = si + 2 * ri, j = sj + 2 * (t - ri * cols);
                    if (flags && !cur[sj * nf + i * WW + (j >> 6)])
                        continue;
                    if (ws_pixel(F, ld, H, W, i, j)) {
                        changed = true;
                        if (flags) {
                            // the words of its neighbours and its own, both parities
                            const int wl = (j > 0 ? j - 1 : 0) >> 6, wr = (j + 1 < W ? j + 1 : j) >> 6;
                            for (int y = i > 0 ? i - 1 : 0; y <= (i + 1 < H ? i + 1 : i); ++y) {
                                nxt[y * WW + wl] = 1;
                                nxt[y * WW + wr] = 1;
                                nxt[nf + y * WW + wl] = 1;
                                nxt[nf + y * WW + wr] = 1;
                            }
                        }
                    }
                }
                if (changed)
                    s_flag = 1;
                // the pass's stores (pixels and flags) before they are read
                __threadfence_block();
                __syncthreads();
                if (flags) {
                    for (int q = threadIdx.x; q < nf; q += WS_NT) {
                        const int row = q / WW;
                        for (int c = 0; c < 2; ++c) {
                            const int k = c * nf + q;
                            // this pass consumed its own flags; the others keep theirs
                            cur[k] = (c == sj && (row & 1) == si) ? nxt[k] : (uint8_t)(cur[k] | nxt[k]);
                            nxt[k] = 0;
                        }
                    }
                    __syncthreads();
                }
            }
            const int any = s_flag;
            __syncthreads();
            if (!any)
                break;
        }
    }
}

namespace hasf_detail {

size_t wshed_lds_bytes(int H, int W)
{
    return 4 * (size_t)H * (size_t)((W + 63) / 64);
}

size_t wshed_lds_max()
{
    return WS_FLAG_BYTES_MAX;
}

hipError_t launch_wshed(const GreyDesc* d_desc, int n, int* d_next, int grid, size_t lds, hipStream_t stream)
{
    static std::atomic<uint64_t> attr{0};
    const hipError_t e = allow_dyn_lds((const void*)hasf_wshed_kernel, (int)WS_FLAG_BYTES_MAX, attr);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(hasf_wshed_kernel, dim3(grid), dim3(WS_NT), lds, stream, d_desc, n, d_next);
    return hipGetLastError();
}

}  // namespace hasf_detail
