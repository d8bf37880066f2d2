// Standalone constrained thinning H(X, K) and thickening *H(Y, V) (Sec. 2)
// with exact priorities: the squared Euclidean distance to the background
// (thinning, outside of the window included) or to Y (thickening), computed
// once by the exact transform before the first level.
//
// One workgroup runs the whole schedule. The distinct priority values of the
// candidates are the levels: they are ranked with a bitmap over the value
// range and a prefix popcount, the candidates are bucketed by rank (counting
// sort), and the levels are then processed in increasing order with the same
// subfield rounds as the filter.
#include "hasf_device.h"

using namespace hasf_dev;


using hasf_detail::TopoArgs;

// threads of the one workgroup that runs a standalone thinning or thickening
constexpr int TOPO_BLOCK = 1024;

namespace {

typedef __attribute__((address_space(1))) uint32_t g32;

// exclusive scan of per-thread values over the block; returns the total
__device__ unsigned block_exclusive_scan(unsigned v, unsigned* out_prefix, unsigned* lds_tmp)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        lds_tmp[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int w = 0; w < TOPO_BLOCK / 64; ++w) {
            const unsigned t = lds_tmp[w];
            lds_tmp[w] = acc;
            acc += t;
        }
        lds_tmp[TOPO_BLOCK / 64] = acc;
    }
    __syncthreads();
    *out_prefix = lds_tmp[wave] + x - v;
    const unsigned total = lds_tmp[TOPO_BLOCK / 64];
    __syncthreads();
    return total;
}

// bit (i, j) of a row-major plane
template <typename PP>
__device__ __forceinline__ bool bit_at(PP plane, int WW, int i, int j)
{
    return (plane[i * WW + (j >> 6)] >> (j & 63)) & 1ull;
}

template <bool LDS>
__device__ void topo_run(const TopoArgs& a, uint64_t* smem)
{
    __shared__ unsigned tmp[TOPO_BLOCK / 64 + 1];
    __shared__ int ctl[CTL_LDS_WORDS];
    Img<LDS> g;
    g.ctl = (lds_i32*)ctl;
    g.H = a.H;
    g.W = a.W;
    glb_u8* gp = (glb_u8*)a.planes;
    size_t boff = 0;
    if constexpr (LDS) {
        bind_state(g, (void*)smem);
    } else {
        bind_state(g, (void*)gp);
        boff = (state_bytes(a.H, a.W, false) + 255) / 256 * 256;
    }
    glb_u64* Bp = (glb_u64*)(gp + boff);  // row-major bits of B
    g.A = nullptr;
    g.K = nullptr;
    g.Dp = nullptr;
    g.hasK = false;
    g.hasD = false;
    g.conn4 = a.conn4 != 0;
    g.eidx = nullptr;
    g.emsk = nullptr;
    const int N = a.H * a.W;
    const int WW = g.WW;

    // X -> R, B -> Bp (row-major); R is read below until the sub-images are built
    pack_rows(a.X, (const uint8_t*)nullptr, a.ld, a.H, a.W, g.R, (glb_u64*)nullptr, threadIdx.x, TOPO_BLOCK);
    if (a.B)
        pack_rows(a.B, (const uint8_t*)nullptr, a.ld, a.H, a.W, Bp, (glb_u64*)nullptr, threadIdx.x, TOPO_BLOCK);
    else
        for (int q = threadIdx.x; q < g.NWD; q += TOPO_BLOCK)
            Bp[q] = 0;
    glb_u64* bm = (glb_u64*)a.bitmap;
    for (unsigned long long q = threadIdx.x; q < a.nbw; q += TOPO_BLOCK)
        bm[q] = 0;
    __syncthreads();

    // mark the priority values of the candidates
    for (int p = threadIdx.x; p < N; p += TOPO_BLOCK) {
        const int i = p / a.W, j = p - i * a.W;
        const bool s = bit_at(g.R, WW, i, j), b = bit_at(Bp, WW, i, j);
        if (a.thin ? (s && !b) : (!s && b)) {
            const uint32_t v = a.P[(size_t)i * a.W + j];
            if (v != 0xFFFFFFFFu)
                __hip_atomic_fetch_or(bm + (v >> 6), 1ull << (v & 63), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();

    // rank base of every bitmap word (prefix popcount, chunked per thread)
    const unsigned long long chunk = (a.nbw + TOPO_BLOCK - 1) / TOPO_BLOCK;
    const unsigned long long c0 = threadIdx.x * chunk, c1 = min(a.nbw, c0 + chunk);
    unsigned local = 0;
    for (unsigned long long q = c0; q < c1; ++q)
        local += __popcll(bm[q]);
    unsigned pre;
    const unsigned nlev = block_exclusive_scan(local, &pre, tmp);
    g32* rb = (g32*)a.rank_base;
    for (unsigned long long q = c0; q < c1; ++q) {
        rb[q] = pre;
        pre += __popcll(bm[q]);
    }
    g32* hist = (g32*)a.hist;
    for (unsigned k = threadIdx.x; k < nlev; k += TOPO_BLOCK)
        hist[k] = 0;
    __syncthreads();

    // count candidates per level
    for (int p = threadIdx.x; p < N; p += TOPO_BLOCK) {
        const int i = p / a.W, j = p - i * a.W;
        const bool s = bit_at(g.R, WW, i, j), b = bit_at(Bp, WW, i, j);
        if (a.thin ? (s && !b) : (!s && b)) {
            const uint32_t v = a.P[(size_t)i * a.W + j];
            if (v != 0xFFFFFFFFu) {
                const uint64_t w = bm[v >> 6];
                const unsigned rk = rb[v >> 6] + __popcll(w & ((1ull << (v & 63)) - 1ull));
                __hip_atomic_fetch_add(hist + rk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    // exclusive offsets per level
    {
        const unsigned long long hc = (nlev + TOPO_BLOCK - 1) / TOPO_BLOCK;
        const unsigned long long h0 = threadIdx.x * hc, h1 = min((unsigned long long)nlev, h0 + hc);
        unsigned loc = 0;
        for (unsigned long long k = h0; k < h1; ++k)
            loc += hist[k];
        unsigned hp;
        block_exclusive_scan(loc, &hp, tmp);
        for (unsigned long long k = h0; k < h1; ++k) {
            const unsigned c = hist[k];
            hist[k] = hp;
            hp += c;
        }
    }
    __syncthreads();
    // scatter: afterwards hist[k] is the end of level k
    g32* ent = (g32*)a.ent;
    for (int p = threadIdx.x; p < N; p += TOPO_BLOCK) {
        const int i = p / a.W, j = p - i * a.W;
        const bool s = bit_at(g.R, WW, i, j), b = bit_at(Bp, WW, i, j);
        if (a.thin ? (s && !b) : (!s && b)) {
            const uint32_t v = a.P[(size_t)i * a.W + j];
            if (v != 0xFFFFFFFFu) {
                const uint64_t w = bm[v >> 6];
                const unsigned rk = rb[v >> 6] + __popcll(w & ((1ull << (v & 63)) - 1ull));
                const unsigned pos = __hip_atomic_fetch_add(hist + rk, 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                ent[pos] = (uint32_t)p;
            }
        }
    }
    __syncthreads();
    rows_to_sub(g, threadIdx.x, TOPO_BLOCK);
    __syncthreads();
    clear_candidates(g, threadIdx.x, TOPO_BLOCK);  // R is no longer needed
    Sched sc;
    sched_reset(g, sc);
    __syncthreads();

    // levels in increasing order
    for (unsigned k = 0; k < nlev; ++k) {
        const unsigned e0 = k ? hist[k - 1] : 0u, e1 = hist[k];
        const int ser = ++sc.serial;
        for (unsigned t = e0 + threadIdx.x; t < e1; t += TOPO_BLOCK) {
            const unsigned p = ent[t];
            const int i = (int)(p / (unsigned)a.W), j = (int)(p - (unsigned)i * (unsigned)a.W);
            activate_pixel(g, i, j, ser);
        }
        __syncthreads();
        run_rounds<LDS, TOPO_BLOCK>(g, a.thin != 0, sc);
    }
    __syncthreads();
    sub_to_rows(g, threadIdx.x, TOPO_BLOCK);
    __syncthreads();
    unpack_rows(a.X, a.ld, a.H, a.W, g.R, threadIdx.x, TOPO_BLOCK);
}

}  // namespace

__global__ __launch_bounds__(TOPO_BLOCK) void hasf_topo_kernel(TopoArgs a)
{
    extern __shared__ uint64_t smem[];
    if (a.lds)
        topo_run<true>(a, smem);
    else
        topo_run<false>(a, smem);
}

namespace hasf_detail {

hipError_t launch_topo(const TopoArgs& a, size_t lds_bytes, hipStream_t stream)
{
    static std::atomic<uint64_t> attr_done{0};
    const hipError_t e = allow_dyn_lds((const void*)hasf_topo_kernel, 160 * 1024 - 4096, attr_done);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(hasf_topo_kernel, dim3(1), dim3(TOPO_BLOCK), lds_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace hasf_detail
