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

// hasf_filter_kernel is built for BLOCK (512) and for this many threads
constexpr int FILTER_BLOCK_MAX = 1024;

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
    g.Dp = g.K + NWD;
    g.hasK = dp->C != nullptr;
    g.hasD = dp->D != nullptr;
    g.conn4 = dp->conn4 != 0;
    g.eidx = (glb_u32*)dp->ent_idx;
    g.emsk = (glb_u64*)dp->ent_msk;
    return g;
}

// Level entry counts: in LDS for a workgroup's image, in global memory for an
// image shared by a grid of workgroups.
template <bool GRID>
using CntPtr = typename std::conditional<GRID, glb_u32*, lds_u32*>::type;

// Append `acc` (candidate bits of row-major word (row, w) at level `rank`) to
// the level's entry list, one atomic per wave. A word has at most one entry
// per level, so a slot never reaches NWD; the bound is checked all the same.
template <bool LDS, bool GRID>
__device__ __forceinline__ void flush_level(const Img<LDS>& g, CntPtr<GRID> cnt, int rank, int row, int w,
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
                                      GRID ? __HIP_MEMORY_SCOPE_AGENT : __HIP_MEMORY_SCOPE_WORKGROUP);
    base = __shfl(base, leader);
    if (acc) {
        const unsigned slot = base + (unsigned)__popcll(pred & lanemask_lt());
        if (slot < (unsigned)g.NWD) {
            const size_t e = (size_t)rank * g.NWD + slot;
            g.eidx[e] = ((uint32_t)row << 10) | (uint32_t)w;
            g.emsk[e] = acc;
        }
    }
}

// One distance/threshold/level stage at radius I, over all words: computes
// the candidate bits of each level of the phase and appends them to the
// level entry lists. Threads t0, t0 + tn, ... share the words (tn is a
// multiple of the wave size).
template <int I, bool LDS, bool GRID>
__device__ __attribute__((noinline)) void stage(const ImgDesc* __restrict__ dp, uint64_t* smem, int mode,
                                                CntPtr<GRID> cnt, lds_i32* ctl, int t0, int tn)
{
    const Img<LDS> g = make_img<LDS>(dp, smem, ctl);
    constexpr BallPairs P = make_ball_pairs(I);
    const bool frame = (mode == HC_THIN || mode == HF_THIN);
    // all lanes of a wave iterate the same number of times so that the
    // wave-level flush sees every lane
    const int nq = (g.NWD + tn - 1) / tn * tn;
    for (int q = t0; q < nq; q += tn) {
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
                // the filling never adds a point of the background constraint
                base = ~s & valid & ~(g.hasD ? g.Dp[q] : 0ull);
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
                flush_level<LDS, GRID>(g, cnt, P.rank[k], row, w, acc);
                acc = 0;
            }
        }
    }
}

template <bool LDS, bool GRID>
__device__ __forceinline__ void run_stage(const ImgDesc* dp, uint64_t* smem, int i, int mode, CntPtr<GRID> cnt,
                                          lds_i32* ctl, int t0, int tn)
{
    switch (i) {
    case 1: stage<1, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 2: stage<2, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 3: stage<3, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 4: stage<4, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 5: stage<5, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 6: stage<6, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 7: stage<7, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 8: stage<8, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 9: stage<9, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 10: stage<10, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 11: stage<11, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 12: stage<12, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 13: stage<13, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    case 14: stage<14, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    default: stage<15, LDS, GRID>(dp, smem, mode, cnt, ctl, t0, tn); break;
    }
}

// Levels in increasing order; inside a level, rounds of the four subfield
// passes until a round changes nothing (the schedule of thinning H and
// thickening *H, Sec. 2).
template <bool LDS, int NT>
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
        for (unsigned t = threadIdx.x; t < c; t += NT) {
            const uint32_t p = g.eidx[e0 + t];
            activate_row_word(g, (int)(p >> 10), (int)(p & 1023u), (uint64_t)g.emsk[e0 + t], ser);
        }
        __syncthreads();
        run_rounds<LDS, NT>(g, thin, sc);
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

template <bool LDS, int NT>
__device__ __attribute__((noinline)) void run_image(const ImgDesc* __restrict__ dp, uint64_t* smem, lds_u32* cnt,
                                                    lds_i32* ctl)
{
    const Img<LDS> g = make_img<LDS>(dp, smem, ctl);
    pack_rows(dp->X, dp->C, dp->ld, g.H, g.W, g.R, g.hasK ? g.K : nullptr, threadIdx.x, NT);
    if (g.hasD)
        pack_background(dp->D, dp->ld, g.H, g.W, g.R, g.Dp, threadIdx.x, NT);
    for (int k = threadIdx.x; k < HASF_LEVELS_MAX; k += NT)
        cnt[k] = 0;
    __syncthreads();
    rows_to_sub(g, threadIdx.x, NT);
    __syncthreads();
    const int r = dp->r;
    // phases in the order of the enum (HC_i then HF_i), or rotated by two for
    // the dual order (HF_i then HC_i); each operator saves its own input in A
    const int rot = dp->order ? 2 : 0;
    for (int i = 1; i <= r; ++i) {
        const int nlev = levels_at(i);
        // HC_i (eq. i): thin, then thicken; HF_i (eq. ii): thicken, then thin
        for (int k = 0; k < 4; ++k) {
            const int ph = (k + rot) & 3;
            if (i > 1 || k > 0) {
                sub_to_rows(g, threadIdx.x, NT);
                __syncthreads();
            }
            run_stage<LDS, false>(dp, smem, i, ph, cnt, ctl, threadIdx.x, NT);
            __syncthreads();
            clear_candidates(g, threadIdx.x, NT);
            __syncthreads();
            level_loop<LDS, NT>(dp, smem, ph == HC_THIN || ph == HF_THIN, nlev, cnt, ctl);
            for (int k = threadIdx.x; k < nlev; k += NT)
                cnt[k] = 0;
            __syncthreads();
        }
    }
    if (r > 0) {
        sub_to_rows(g, threadIdx.x, NT);
        __syncthreads();
    }
    unpack_rows(dp->X, dp->ld, g.H, g.W, g.R, threadIdx.x, NT);
}

// ---------------------------------------------------------------------------
// One large image shared by a grid of workgroups. The state is in global
// memory; every step runs over the whole grid (thread t0 of tn takes words
// t0, t0 + tn, ...) and the workgroup barriers of the per-image kernel become
// grid barriers. A subfield pass tests its flagged words directly (no live
// list), so it takes one grid barrier.
// ---------------------------------------------------------------------------
struct GridSync {
    GridCtl* gc;
    unsigned nblk;
    unsigned gen;     // grid barriers completed: the current epoch, uniform over the grid
    unsigned rounds;  // rounds of the level loops (uniform)
    unsigned acts;    // levels activated (uniform)
};

// a grid barrier that waits longer than this (100 MHz ticks: 4 s) gives up
constexpr unsigned long long GRID_WAIT_LIMIT = 400000000ull;

// Pass control words (chg, prod[4]) by epoch parity: during epoch e every
// workgroup reads copy e & 1 and writes copy (e + 1) & 1, so the decisions of
// an epoch (skip a pass, end a round) never see a value written in the same
// epoch by a faster workgroup. Written values are serials, larger than any
// before them; at the start of each epoch workgroup 0 carries the read copy
// into the written one with atomic max, so the next epoch reads the whole
// history. The read copy of an epoch is loaded once (CtlView).
struct CtlView {
    int w[CTL_WORDS];
};

__device__ __forceinline__ CtlView ctl_view(const GridSync& gs)
{
    CtlView v;
    const int4* p = reinterpret_cast<const int4*>(gs.gc->ctl[gs.gen & 1]);
    const int4 a = p[0], b = p[1];
    v.w[0] = a.x; v.w[1] = a.y; v.w[2] = a.z; v.w[3] = a.w;
    v.w[4] = b.x; v.w[5] = b.y; v.w[6] = b.z; v.w[7] = b.w;
    return v;
}

__device__ __forceinline__ void ctl_wr(const GridSync& gs, int x, int v)
{
    __hip_atomic_store(&gs.gc->ctl[(gs.gen + 1) & 1][x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier. Every wave first waits for its own stores; one thread per
// workgroup then releases them at device scope (L2 write-back), counts the
// workgroup in and waits for the last arrival's generation bump, then
// acquires (L2 invalidate). Waits are bounded: on time-out, or when another
// workgroup has given up, it returns false and the caller returns.
__device__ __forceinline__ bool grid_sync(GridSync& gs, int* s_ok)
{
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
        GridCtl* gc = gs.gc;
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned target = (gs.gen + 1) * gs.nblk;
        const unsigned old = __hip_atomic_fetch_add(&gc->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == target) {
            __hip_atomic_store(&gc->bar_gen, gs.gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(&gc->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gs.gen) {
                if (__hip_atomic_load(&gc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > GRID_WAIT_LIMIT) {
                    __hip_atomic_store(&gc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    ++gs.gen;
    __syncthreads();
    // carry the history into the copy this epoch writes (see CtlView)
    if (blockIdx.x == 0 && threadIdx.x < CTL_WORDS)
        __hip_atomic_fetch_max(&gs.gc->ctl[(gs.gen + 1) & 1][threadIdx.x], gs.gc->ctl[gs.gen & 1][threadIdx.x],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *s_ok != 0;
}

// flagged words a workgroup lists per chunk of a pass: GRID_CHUNK flag
// words (4 bytes each) per thread
constexpr int GRID_CHUNK = 4;
constexpr int GRID_LIST = GRID_CHUNK * 4 * BLOCK;

// exclusive prefix over the wave of v in [0, 31]; *total = sum over the wave
__device__ __forceinline__ unsigned wave_prefix32(unsigned v, unsigned* total)
{
    const uint64_t lt = lanemask_lt();
    unsigned pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const uint64_t m = __ballot((v >> b) & 1u);
        pre += (unsigned)__popcll(m & lt) << b;
        tot += (unsigned)__popcll(m) << b;
    }
    *total = tot;
    return pre;
}

// Rounds of the four subfield passes until a round changes nothing (the same
// schedule as run_rounds). A pass goes over its sub-image in chunks: each
// thread loads GRID_CHUNK flag words at once (interleaved over the grid) and
// lists its flagged words in the workgroup's LDS list; after a workgroup
// barrier the list is tested densely, each word's loads issued together.
// This keeps a pass at about two dependent global round trips.
__device__ __forceinline__ bool rounds_grid(const Img<false>& g, GridSync& gs, int* s_ok, bool thin, Sched& sc,
                                            int t0, int tn, lds_u32* list, lds_u32* lcount)
{
    const uint32_t flip = thin ? 0u : ~0u;
    CtlView v = ctl_view(gs);
    for (;;) {
        ++gs.rounds;
        const int round_start = sc.serial;
        for (int s = 0; s < 4; ++s) {
            const int p = v.w[CTL_PROD + s];
            if (p <= sc.consumed[s])
                continue;
            sc.consumed[s] = p;
            const int ser = ++sc.serial;
            const int si = s >> 1, sj = s & 1;
            const int so = 1 - si, co = 1 - sj;
            const PassPtrs<false> pp = pass_ptrs(g, si, sj);
            glb_u32* D4 = (glb_u32*)(g.D + g.sub(si, sj));
            const int nw = ((g.H - si + 1) >> 1) * g.WW;
            const int nw4 = (nw + 3) >> 2;
            const int nchunk = (nw4 + GRID_CHUNK * tn - 1) / (GRID_CHUNK * tn);  // uniform
            bool changed = false;
            for (int ch = 0; ch < nchunk; ++ch) {
                // the four words' M and S come with their flags (one round
                // trip), so only flagged words with live candidates are listed
                // (4 * q4 + 3 < roundup4(nw) <= SUB: in the sub-image)
                uint32_t f4[GRID_CHUNK];
                u32x4 m4[GRID_CHUNK], s4[GRID_CHUNK];
#pragma unroll
                for (int k = 0; k < GRID_CHUNK; ++k) {
                    const int q4 = t0 + (ch * GRID_CHUNK + k) * tn;
                    f4[k] = 0u;
                    m4[k] = s4[k] = u32x4{0u, 0u, 0u, 0u};
                    if (q4 < nw4) {
                        f4[k] = D4[q4];
                        m4[k] = *(const glb_u4*)(pp.Ms + 4 * q4);
                        s4[k] = *(const glb_u4*)(pp.Ss + 4 * q4);
                    }
                }
                unsigned nl = 0;
#pragma unroll
                for (int k = 0; k < GRID_CHUNK; ++k) {
                    if (f4[k]) {
                        const int q0 = 4 * (t0 + (ch * GRID_CHUNK + k) * tn);
                        D4[t0 + (ch * GRID_CHUNK + k) * tn] = 0u;
                        uint32_t keep = 0u;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (((f4[k] >> (8 * j)) & 0xFFu) && q0 + j < nw && (m4[k][j] & (s4[k][j] ^ flip)))
                                keep |= 1u << (8 * j);
                        f4[k] = keep;
                        nl += __popc(keep);
                    }
                }
                // list counts alternate between chunks (sc.npass counts them);
                // the other one is cleared once every thread has read it
                const int cc = sc.npass++;
                lds_u32* cnt = lcount + (cc & 1);
                unsigned tot;
                const unsigned off = wave_prefix32(nl, &tot);
                unsigned base = 0;
                if (tot) {
                    if ((threadIdx.x & 63) == 0)
                        base = __hip_atomic_fetch_add(cnt, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    base = (unsigned)__builtin_amdgcn_readfirstlane((int)base) + off;
#pragma unroll
                    for (int k = 0; k < GRID_CHUNK; ++k) {
                        const int q0 = 4 * (t0 + (ch * GRID_CHUNK + k) * tn);
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if ((f4[k] >> (8 * j)) & 1u)
                                list[base++] = (uint32_t)(q0 + j);
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0)
                    lcount[(cc + 1) & 1] = 0u;
                const int n = (int)*cnt;
                for (int t = threadIdx.x; t < n; t += BLOCK) {
                    const int q = (int)list[t];
                    if (q < nw)
                        changed |= test_word(pp, q, q / g.WW, si, sj, g.WW, g.H, flip, g.conn4);
                }
                if (ch + 1 < nchunk)
                    __syncthreads();  // the next chunk rewrites the list (the grid barrier ends the last)
            }
            const uint64_t chm = __ballot(changed);
            if (chm && (int)(threadIdx.x & 63) == __ffsll((long long)chm) - 1) {
                ctl_wr(gs, CTL_CHG, ser);
                ctl_wr(gs, CTL_PROD + si * 2 + co, ser);
                if (g.H > 1) {
                    ctl_wr(gs, CTL_PROD + so * 2 + sj, ser);
                    ctl_wr(gs, CTL_PROD + so * 2 + co, ser);
                }
            }
            if (!grid_sync(gs, s_ok))
                return false;
            v = ctl_view(gs);
        }
        if (v.w[CTL_CHG] <= round_start)
            break;
    }
    return true;
}

// Levels in increasing order, as level_loop; the caller has cleared the
// candidates and the control words.
__device__ __forceinline__ bool level_loop_grid(const Img<false>& g, GridSync& gs, int* s_ok, bool thin, int nlev,
                                                int t0, int tn, lds_u32* list, lds_u32* lcount)
{
    Sched sc;
    sc.serial = 0;
    sc.npass = 0;  // here: chunks listed so far (selects the list count)
    for (int k = 0; k < 4; ++k)
        sc.consumed[k] = 0;
    if (threadIdx.x == 0)
        lcount[0] = lcount[1] = 0u;
    __syncthreads();
    for (int k = 0; k < nlev; ++k) {
        const unsigned c = min(__hip_atomic_load(&gs.gc->cnt[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                               (unsigned)g.NWD);
        if (c == 0)
            continue;
        const int ser = ++sc.serial;
        ++gs.acts;
        const size_t e0 = (size_t)k * g.NWD;
        unsigned touched = 0;  // bit s: a word of sub-image s was activated
        for (unsigned t = t0; t < c; t += tn) {
            const uint32_t pe = g.eidx[e0 + t];
            const int row = (int)(pe >> 10), w = (int)(pe & 1023u);
            if (row >= g.H || w >= g.WW)
                continue;
            const uint64_t m = g.emsk[e0 + t];
            const int o = (row >> 1) * g.WW + w;
            const uint32_t ev = even_bits(m), od = even_bits(m >> 1);
            if (ev) {
                const int q = g.sub(row & 1, 0) + o;
                __hip_atomic_fetch_or(g.M + q, ev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                g.D[q] = 1;
                touched |= 1u << ((row & 1) * 2);
            }
            if (od) {
                const int q = g.sub(row & 1, 1) + o;
                __hip_atomic_fetch_or(g.M + q, od, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                g.D[q] = 1;
                touched |= 1u << ((row & 1) * 2 + 1);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (__ballot((touched >> b) & 1u) && (threadIdx.x & 63) == 0)
                ctl_wr(gs, CTL_PROD + b, ser);
        if (!grid_sync(gs, s_ok))
            return false;
        if (!rounds_grid(g, gs, s_ok, thin, sc, t0, tn, list, lcount))
            return false;
    }
    return true;
}

// The whole filter on one image, over the grid (as run_image).
__device__ __forceinline__ bool run_image_grid(const ImgDesc* __restrict__ dp, GridCtl* gc, int* s_ok,
                                               lds_u32* list, lds_u32* lcount, GridSync& gs)
{
    const int t0 = blockIdx.x * BLOCK + threadIdx.x, tn = gridDim.x * BLOCK;
    const Img<false> g = make_img<false>(dp, nullptr, nullptr);
    pack_rows(dp->X, dp->C, dp->ld, g.H, g.W, g.R, g.hasK ? g.K : nullptr, t0, tn);
    if (g.hasD)
        pack_background(dp->D, dp->ld, g.H, g.W, g.R, g.Dp, t0, tn);
    if (!grid_sync(gs, s_ok))
        return false;
    rows_to_sub(g, t0, tn);
    if (!grid_sync(gs, s_ok))
        return false;
    const int r = dp->r;
    const int rot = dp->order ? 2 : 0;  // as in run_image
    for (int i = 1; i <= r; ++i) {
        const int nlev = levels_at(i);
        for (int k = 0; k < 4; ++k) {
            const int ph = (k + rot) & 3;
            if (i > 1 || k > 0) {
                sub_to_rows(g, t0, tn);
                if (!grid_sync(gs, s_ok))
                    return false;
            }
            run_stage<false, true>(dp, nullptr, i, ph, (glb_u32*)gc->cnt, nullptr, t0, tn);
            if (!grid_sync(gs, s_ok))
                return false;
            clear_candidates(g, t0, tn);
            // the threads that carried the control words at the start of this
            // epoch clear both copies (no pass reads or writes them now)
            if (blockIdx.x == 0 && threadIdx.x < CTL_WORDS) {
                __hip_atomic_store(&gc->ctl[0][threadIdx.x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&gc->ctl[1][threadIdx.x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!grid_sync(gs, s_ok))
                return false;
            if (!level_loop_grid(g, gs, s_ok, ph == HC_THIN || ph == HF_THIN, nlev, t0, tn, list, lcount))
                return false;
            // every workgroup has read the counts of the levels it ran (a
            // workgroup still finishing its last round only reads zeros)
            if (blockIdx.x == 0)
                for (int k = threadIdx.x; k < nlev; k += BLOCK)
                    __hip_atomic_store(&gc->cnt[k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (r > 0) {
        sub_to_rows(g, t0, tn);
        if (!grid_sync(gs, s_ok))
            return false;
    }
    unpack_rows(dp->X, dp->ld, g.H, g.W, g.R, t0, tn);
    return true;
}

}  // namespace

// One image over the whole grid. If a grid barrier gave up, gc->err and the
// caller's sticky word *err_out are set (the image is then undefined).
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void hasf_grid_kernel(
    const ImgDesc* __restrict__ dp, GridCtl* gc, unsigned* err_out)
{
    __shared__ int s_ok;
    __shared__ uint32_t list[GRID_LIST];
    __shared__ uint32_t lcount[2];
    GridSync gs{gc, gridDim.x, 0u, 0u, 0u};
    const bool ok = run_image_grid(dp, gc, &s_ok, (lds_u32*)list, (lds_u32*)lcount, gs);
    if (!ok && threadIdx.x == 0) {
        __hip_atomic_store(&gc->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (err_out)
            __hip_atomic_fetch_or(err_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the schedule's counts (uniform over the grid: workgroup 0 reports them)
    if (ok && err_out && blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned long long* c = reinterpret_cast<unsigned long long*>(err_out + GRID_COUNTS_OFF);
        __hip_atomic_fetch_add(c + 0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 1, (unsigned long long)gs.rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 2, (unsigned long long)gs.acts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 3, (unsigned long long)gs.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Each workgroup claims images in queue order until the queue is empty. When
// `done` is given (host-mapped memory), done[q] becomes 1 once image q's
// result is in memory, so the host can hand it out before the launch ends.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void hasf_filter_kernel(
    const ImgDesc* __restrict__ desc, int n, int* __restrict__ next, unsigned* done)
{
    extern __shared__ uint64_t smem[];
    __shared__ unsigned cnt[HASF_LEVELS_MAX];
    __shared__ int ctl[CTL_LDS_WORDS];
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
            run_image<true, NT>(desc + img, smem, (lds_u32*)cnt, (lds_i32*)ctl);
        else
            run_image<false, NT>(desc + img, smem, (lds_u32*)cnt, (lds_i32*)ctl);
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

// Workgroup size of a launch of n images: with at most one image per CU,
// 1024 threads per image (a lone image finishes sooner with more waves);
// beyond that 512, so that two images share a CU and hide each other's
// barrier stalls (measured on 512x512 r=5: 1024 images at 512 threads
// 117 K frames/s against 83 K at 1024; one image 2.8 ms against 3.3 ms).
int filter_block_for(int n, int num_cu)
{
    return n <= num_cu ? FILTER_BLOCK_MAX : BLOCK;
}

hipError_t launch_filter(const ImgDesc* d_desc, int n, int* d_next, int grid, int block, size_t lds_bytes,
                         hipStream_t stream, unsigned* done)
{
    static std::atomic<uint64_t> attr_512{0}, attr_1024{0};
    hipError_t e;
    if (block == FILTER_BLOCK_MAX) {
        e = allow_dyn_lds((const void*)hasf_filter_kernel<FILTER_BLOCK_MAX>, 160 * 1024 - 2048, attr_1024);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(hasf_filter_kernel<FILTER_BLOCK_MAX>, dim3(grid), dim3(block), lds_bytes, stream, d_desc,
                           n, d_next, done);
    } else {
        e = allow_dyn_lds((const void*)hasf_filter_kernel<BLOCK>, 160 * 1024 - 2048, attr_512);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(hasf_filter_kernel<BLOCK>, dim3(grid), dim3(BLOCK), lds_bytes, stream, d_desc, n,
                           d_next, done);
    }
    return hipGetLastError();
}

}  // namespace hasf_detail

namespace hasf_detail {

hipError_t launch_grid(const ImgDesc* d_desc, GridCtl* d_ctl, unsigned* d_err, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(hasf_grid_kernel, dim3(grid), dim3(BLOCK), 0, stream, d_desc, d_ctl, d_err);
    return hipGetLastError();
}

int grid_occupancy()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, hasf_grid_kernel, BLOCK, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

int filter_occupancy(size_t lds_bytes, int block)
{
    int blocks = 0;
    const hipError_t e = block == FILTER_BLOCK_MAX
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                   &blocks, hasf_filter_kernel<FILTER_BLOCK_MAX>, block, lds_bytes)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, hasf_filter_kernel<BLOCK>,
                                                                            BLOCK, lds_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

}  // namespace hasf_detail

