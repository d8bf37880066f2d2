// Persistent per-image HASF kernel for gfx950.
//
// One workgroup (512 threads, 8 wave64s) owns one image at a time and runs
// the whole radius loop of the filter on it (Sec. 2: HASF = HF_r o HC_r o ...
// o HF_1 o HC_1), so every synchronisation of the level/round/subfield
// schedule is a workgroup barrier. Workgroups claim images from a queue
// (atomic counter over a descriptor array sorted by decreasing cost).
//
// State is bit-packed: one bit per pixel, 64 pixels of a row per 64-bit word,
// bit p of word w = column 64w + p. Planes:
//   S  the current set                      (LDS when it fits, else global)
//   M  activated candidates of the phase    (LDS when it fits, else global)
//   A  the set saved before a phase         (global)
//   K  the constraint set C n X             (global)
//
// Distances. Inside the filter a distance map is only ever compared with i^2
// for the current radius i (ball thresholds) or used to order candidates
// whose distance is <= i^2. So the squared distance of a pixel is only needed
// when it is <= i^2, and it is obtained from the ball offsets (a, b) sorted by
// a^2 + b^2: with V_a = rows within +-a of the features (vertical dilation),
// the pixels first reached by V_a shifted by +-b have squared distance
// a^2 + b^2 exactly. This is evaluated on whole words, per level, and
// produces the candidate bits of each level directly as (word, mask) entries.
#include <atomic>

#include "hasf_device.h"

using namespace hasf_dev;

namespace {

// Feature word at (row, w) for the distance map of this stage.
// frame: features = complement of S plus everything outside the window.
template <bool LDS>
__device__ __forceinline__ uint64_t feat_word(const Img<LDS>& g, int row, int w, bool frame)
{
    if (row < 0 || row >= g.H || w < 0 || w >= g.WW)
        return frame ? ~0ull : 0ull;
    const uint64_t s = g.R[row * g.WW + w];
    return frame ? ~s : s;  // bits past W: ~0 = outside (frame) / 0 (no frame)
}

template <bool LDS>
__device__ __forceinline__ Img<LDS> make_img(const ImgDesc* __restrict__ dp, uint64_t* smem, lds_i32* ctl)
{
    Img<LDS> g;
    g.ctl = ctl;
    g.H = dp->H;
    g.W = dp->W;
    glb_u64* gp = (glb_u64*)dp->gplanes;
    const size_t NWD = (size_t)g.H * ((g.W + 63) >> 6);
    if constexpr (LDS) {
        bind_state(g, (void*)smem);
        g.A = gp;
        g.K = gp + NWD;
    } else {
        bind_state(g, (void*)gp);
        const size_t sb = (state_bytes(g.H, g.W, false) + 255) / 256 * 256;
        g.A = (glb_u64*)((glb_u8*)gp + sb);
        g.K = g.A + NWD;
    }
    g.hasK = dp->C != nullptr;
    g.eidx = (glb_u32*)dp->ent_idx;
    g.emsk = (glb_u64*)dp->ent_msk;
    return g;
}

// Append `acc` (candidate bits of row-major word (row, w) at level `rank`) to
// the level's entry list, one LDS atomic per wave.
template <bool LDS>
__device__ __forceinline__ void flush_level(const Img<LDS>& g, lds_u32* cnt, int rank, int row, int w,
                                            uint64_t acc)
{
    const uint64_t pred = __ballot(acc != 0);
    if (pred == 0)
        return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)pred) - 1;
    unsigned base = 0;
    if (lane == leader)
        base = __hip_atomic_fetch_add(cnt + rank, (unsigned)__popcll(pred), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    base = __shfl(base, leader);
    if (acc) {
        const unsigned slot = base + (unsigned)__popcll(pred & lanemask_lt());
        const size_t e = (size_t)rank * g.NWD + slot;
        g.eidx[e] = ((uint32_t)row << 10) | (uint32_t)w;
        g.emsk[e] = acc;
    }
}

// One distance/threshold/level stage at radius I, over all words: computes
// the candidate bits of each level of the phase and appends them to the
// level entry lists.
template <int I, bool LDS>
__device__ __attribute__((noinline)) void stage(const ImgDesc* __restrict__ dp, uint64_t* smem, int mode,
                                                lds_u32* cnt, lds_i32* ctl)
{
    const Img<LDS> g = make_img<LDS>(dp, smem, ctl);
    constexpr BallPairs P = make_ball_pairs(I);
    const bool frame = (mode == HC_THIN || mode == HF_THIN);
    // all lanes of a wave iterate the same number of times so that the
    // wave-level flush sees every lane
    const int nq = (g.NWD + BLOCK - 1) / BLOCK * BLOCK;
    for (int q = threadIdx.x; q < nq; q += BLOCK) {
        uint64_t base = 0;
        int row = 0, w = 0;
        if (q < g.NWD) {
            row = q / g.WW;
            w = q - row * g.WW;
            const uint64_t s = g.R[q];
            const uint64_t valid = (w == g.WW - 1) ? g.lastmask : ~0ull;
            switch (mode) {
            case HC_THIN:
                base = s & ~(g.hasK ? g.K[q] : 0ull);
                g.A[q] = s;
                break;
            case HC_THICKEN:
                base = ~s & g.A[q] & valid;
                break;
            case HF_THICKEN:
                base = ~s & valid;
                g.A[q] = s;
                break;
            default:
                base = s & ~g.A[q];
                break;
            }
        }
        if (__ballot(base != 0) == 0)
            continue;  // no candidate in the whole wave
        // Vc[a]: rows within +-a of a feature, this word; E[a]: the same for the
        // 16 columns on each side (low half: top bits of word w-1, high half:
        // low bits of word w+1); shifts never exceed I <= 15 columns.
        uint64_t Vc[I + 1];
        uint32_t E[I + 1];
        {
            uint64_t vm = 0, vc = 0, vp = 0;
            if (base) {
                vm = feat_word(g, row, w - 1, frame);
                vc = feat_word(g, row, w, frame);
                vp = feat_word(g, row, w + 1, frame);
            }
            Vc[0] = vc;
            E[0] = (uint32_t)(vm >> 48) | ((uint32_t)vp << 16);
#pragma unroll
            for (int a = 1; a <= I; ++a) {
                if (base) {
                    vm |= feat_word(g, row - a, w - 1, frame) | feat_word(g, row + a, w - 1, frame);
                    vc |= feat_word(g, row - a, w, frame) | feat_word(g, row + a, w, frame);
                    vp |= feat_word(g, row - a, w + 1, frame) | feat_word(g, row + a, w + 1, frame);
                }
                Vc[a] = vc;
                E[a] = (uint32_t)(vm >> 48) | ((uint32_t)vp << 16);
            }
            if ((Vc[I] | E[I]) == 0)
                base = 0;
        }
        uint64_t cov = 0, acc = 0;
#pragma unroll
        for (int k = 0; k < P.n; ++k) {
            const int a = P.a[k];
            const int b = P.b[k];
            uint64_t x = Vc[a];
            if (b > 0)
                x = (Vc[a] << b) | (uint64_t)((E[a] & 0xFFFFu) >> (16 - b)) | (Vc[a] >> b) |
                    ((uint64_t)(E[a] >> 16) << (64 - b));
            acc |= x & ~cov & base;
            cov |= x;
            if (k == P.n - 1 || P.v[k + 1] != P.v[k]) {
                flush_level(g, cnt, P.rank[k], row, w, acc);
                acc = 0;
            }
        }
    }
}

template <bool LDS>
__device__ __forceinline__ void run_stage(const ImgDesc* dp, uint64_t* smem, int i, int mode, lds_u32* cnt,
                                          lds_i32* ctl)
{
    switch (i) {
    case 1: stage<1, LDS>(dp, smem, mode, cnt, ctl); break;
    case 2: stage<2, LDS>(dp, smem, mode, cnt, ctl); break;
    case 3: stage<3, LDS>(dp, smem, mode, cnt, ctl); break;
    case 4: stage<4, LDS>(dp, smem, mode, cnt, ctl); break;
    case 5: stage<5, LDS>(dp, smem, mode, cnt, ctl); break;
    case 6: stage<6, LDS>(dp, smem, mode, cnt, ctl); break;
    case 7: stage<7, LDS>(dp, smem, mode, cnt, ctl); break;
    case 8: stage<8, LDS>(dp, smem, mode, cnt, ctl); break;
    case 9: stage<9, LDS>(dp, smem, mode, cnt, ctl); break;
    case 10: stage<10, LDS>(dp, smem, mode, cnt, ctl); break;
    case 11: stage<11, LDS>(dp, smem, mode, cnt, ctl); break;
    case 12: stage<12, LDS>(dp, smem, mode, cnt, ctl); break;
    case 13: stage<13, LDS>(dp, smem, mode, cnt, ctl); break;
    case 14: stage<14, LDS>(dp, smem, mode, cnt, ctl); break;
    default: stage<15, LDS>(dp, smem, mode, cnt, ctl); break;
    }
}

// Levels in increasing order; inside a level, rounds of the four subfield
// passes until a round changes nothing (the schedule of thinning H and
// thickening *H, Sec. 2).
template <bool LDS>
__device__ __attribute__((noinline)) void level_loop(const ImgDesc* __restrict__ dp, uint64_t* smem, bool thin,
                                                     int nlev, lds_u32* cnt, lds_i32* ctl)
{
    const Img<LDS> g = make_img<LDS>(dp, smem, ctl);
    Sched sc;
    sched_reset(g, sc);
    __syncthreads();
    for (int k = 0; k < nlev; ++k) {
        const unsigned c = cnt[k];
        if (c == 0)
            continue;
        const int ser = ++sc.serial;
        const size_t e0 = (size_t)k * g.NWD;
        for (unsigned t = threadIdx.x; t < c; t += BLOCK) {
            const uint32_t p = g.eidx[e0 + t];
            activate_row_word(g, (int)(p >> 10), (int)(p & 1023u), (uint64_t)g.emsk[e0 + t], ser);
        }
        __syncthreads();
        run_rounds(g, thin, sc);
    }
    __syncthreads();
}

__device__ int levels_at(int i)
{
    // distinct nonzero sums of two squares <= i^2, i = 0..HASF_R_MAX
    constexpr int tab[HASF_R_MAX + 1] = {
        level_count(0), level_count(1), level_count(2), level_count(3), level_count(4),
        level_count(5), level_count(6), level_count(7), level_count(8), level_count(9),
        level_count(10), level_count(11), level_count(12), level_count(13), level_count(14),
        level_count(15)};
    return tab[i];
}

template <bool LDS>
__device__ __attribute__((noinline)) void run_image(const ImgDesc* __restrict__ dp, uint64_t* smem, lds_u32* cnt,
                                                    lds_i32* ctl)
{
    const Img<LDS> g = make_img<LDS>(dp, smem, ctl);
    pack_rows(dp->X, dp->C, dp->ld, g.H, g.W, g.R, g.hasK ? g.K : nullptr);
    for (int k = threadIdx.x; k < HASF_LEVELS_MAX; k += BLOCK)
        cnt[k] = 0;
    __syncthreads();
    rows_to_sub(g);
    __syncthreads();
    const int r = dp->r;
    for (int i = 1; i <= r; ++i) {
        const int nlev = levels_at(i);
        // HC_i (eq. i): thin, then thicken; HF_i (eq. ii): thicken, then thin
        for (int ph = 0; ph < 4; ++ph) {
            if (i > 1 || ph > 0) {
                sub_to_rows(g);
                __syncthreads();
            }
            run_stage<LDS>(dp, smem, i, ph, cnt, ctl);
            __syncthreads();
            clear_candidates(g);
            __syncthreads();
            level_loop<LDS>(dp, smem, ph == HC_THIN || ph == HF_THIN, nlev, cnt, ctl);
            for (int k = threadIdx.x; k < nlev; k += BLOCK)
                cnt[k] = 0;
            __syncthreads();
        }
    }
    if (r > 0) {
        sub_to_rows(g);
        __syncthreads();
    }
    unpack_rows(dp->X, dp->ld, g.H, g.W, g.R);
}

}  // namespace

// Each workgroup claims images in queue order until the queue is empty. When
// `done` is given (host-mapped memory), done[q] becomes 1 once image q's
// result is in memory, so the host can hand it out before the launch ends.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void hasf_filter_kernel(
    const ImgDesc* __restrict__ desc, int n, int* __restrict__ next, unsigned* done)
{
    extern __shared__ uint64_t smem[];
    __shared__ unsigned cnt[HASF_LEVELS_MAX];
    __shared__ int ctl[CTL_WORDS];
    __shared__ int s_img;
    for (;;) {
        if (threadIdx.x == 0)
            s_img = atomicAdd(next, 1);
        __syncthreads();
        const int img = s_img;
        __syncthreads();
        if (img >= n)
            break;
        if (desc[img].lds)
            run_image<true>(desc + img, smem, (lds_u32*)cnt, (lds_i32*)ctl);
        else
            run_image<false>(desc + img, smem, (lds_u32*)cnt, (lds_i32*)ctl);
        if (done) {
            __threadfence();  // each thread's stores of the image reach device scope
            __syncthreads();
            if (threadIdx.x == 0) {
                // and the whole image is visible to the host and to copy
                // engines before its completion word
                __threadfence_system();
                __hip_atomic_store(done + img, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace hasf_detail {

int filter_block() { return BLOCK; }

hipError_t launch_filter(const ImgDesc* d_desc, int n, int* d_next, int grid, size_t lds_bytes,
                         hipStream_t stream, unsigned* done)
{
    // launched from the caller's thread and from a server's dispatcher thread
    static std::atomic<bool> attr_set{false};
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t e = hipFuncSetAttribute((const void*)hasf_filter_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
        if (e != hipSuccess)
            return e;
        attr_set.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL(hasf_filter_kernel, dim3(grid), dim3(BLOCK), lds_bytes, stream, d_desc, n, d_next, done);
    return hipGetLastError();
}

}  // namespace hasf_detail

namespace hasf_detail {

int filter_occupancy(size_t lds_bytes)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, hasf_filter_kernel, BLOCK, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

}  // namespace hasf_detail

