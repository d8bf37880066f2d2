// One large image filtered by row tiles whose state stays in LDS (the
// schedule of thinning H and thickening *H of Sec. 2, run with temporal
// blocking).
//
// Tile t (one workgroup) owns image rows [t TH, (t + 1) TH) and also keeps
// `halo` rows on each side that its neighbours own, so its LDS state is a
// band of up to TH + 2 halo rows in the layout of the per-image kernel. A
// subfield pass decides a pixel from its 3x3 neighbourhood, so after k passes
// a band's rows can differ from the whole-image schedule only within k rows
// of the band's cut edges: a tile runs halo / 4 rounds (4 passes each, halo
// passes in all) on its own and its own rows are then exactly the
// schedule's. Then every tile publishes its first and last halo own rows,
// the tiles meet at one grid barrier, and each replaces
// its halo rows with its neighbours' (flagging every word whose test reads
// a changed word). A level of the schedule ends after the first round that
// changes nothing anywhere; the tiles learn it at the barrier that follows,
// and the rounds they ran after it changed nothing. So the result is the
// schedule's bit for bit, with one grid barrier per halo / 4 rounds instead
// of one per pass.
//
// Distances: each tile labels the candidates of its whole band from the
// row-major copy of the set in global memory (Rg), which the owners of the
// rows write at the end of every phase, so neighbours label their shared
// rows alike. The saved set A, the constraint K and the background
// constraint Dp are row-major planes in global memory, written by the owners
// of the rows and read by the stages.
#include <atomic>

#include "hasf_device.h"

using namespace hasf_dev;

namespace {

// a grid barrier that waits longer than this (100 MHz ticks: 4 s) gives up
constexpr unsigned long long TILE_WAIT_LIMIT = 400000000ull;

struct TileSync {
    TileCtl* tc;
    unsigned nblk;
    unsigned gen;     // barriers passed (uniform)
    unsigned round;   // rounds run in this launch (uniform)
    unsigned rounds;  // rounds of the schedule (uniform)
    unsigned acts;    // levels activated (uniform)
};

// Grid barrier: every wave waits for its own stores; one thread per
// workgroup releases them at device scope, counts the workgroup in, waits
// for the last arrival's generation bump and acquires. Bounded: on time-out,
// or when another workgroup gave up, it returns false.
__device__ __forceinline__ bool tile_sync(TileSync& ts, int* s_ok)
{
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
        TileCtl* tc = ts.tc;
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned target = (ts.gen + 1) * ts.nblk;
        const unsigned old = __hip_atomic_fetch_add(&tc->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == target) {
            __hip_atomic_store(&tc->bar_gen, ts.gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(&tc->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ts.gen) {
                if (__hip_atomic_load(&tc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > TILE_WAIT_LIMIT) {
                    __hip_atomic_store(&tc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    ++ts.gen;
    __syncthreads();
    return *s_ok != 0;
}

// What a tile's distance stage reads and writes (global rows and words).
struct TileView {
    const glb_u64* Rg;
    glb_u64* A;
    const glb_u64* K;
    const glb_u64* Dp;
    glb_u32* eidx;  // this tile's level entries, `slots` per level
    glb_u64* emsk;
    size_t slots;
    int H, WW;
    uint64_t lastmask;
    int e0, ER, r0, r1;  // band rows [e0, e0 + ER); own rows [r0, r1)
    bool hasK, hasD;
};

__device__ __forceinline__ uint64_t tile_feat(const TileView& v, int row, int w, bool frame)
{
    if (row < 0 || row >= v.H || w < 0 || w >= v.WW)
        return frame ? ~0ull : 0ull;
    const uint64_t s = v.Rg[(size_t)row * v.WW + w];
    return frame ? ~s : s;  // bits past W: ~0 = outside (frame) / 0 (no frame)
}

// Append `acc` (candidate bits of band word (lrow, w) at level `rank`) to the
// tile's entry list of the level, one LDS atomic per wave.
__device__ __forceinline__ void tile_flush(const TileView& v, lds_u32* cnt, int rank, int lrow, int w, uint64_t acc)
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
        if (slot < (unsigned)v.slots) {
            const size_t e = (size_t)rank * v.slots + slot;
            v.eidx[e] = ((uint32_t)lrow << 10) | (uint32_t)w;
            v.emsk[e] = acc;
        }
    }
}

// The distance/threshold/level stage of the per-image kernel at radius I,
// over the words of the tile's band: candidates of the phase labelled with
// their level from the ball offsets (a, b) in increasing a^2 + b^2.
template <int I>
__device__ __attribute__((noinline)) void tile_stage(const TileView& v, int mode, lds_u32* cnt)
{
    constexpr BallPairs P = make_ball_pairs(I);
    const bool frame = (mode == HC_THIN || mode == HF_THIN);
    const int nwb = v.ER * v.WW;
    const int nq = (nwb + TILE_NT - 1) / TILE_NT * TILE_NT;
    for (int q = threadIdx.x; q < nq; q += TILE_NT) {
        uint64_t base = 0;
        int lrow = 0, w = 0, row = 0;
        if (q < nwb) {
            lrow = q / v.WW;
            w = q - lrow * v.WW;
            row = v.e0 + lrow;
            const size_t gq = (size_t)row * v.WW + w;
            const uint64_t s = v.Rg[gq];
            const uint64_t valid = (w == v.WW - 1) ? v.lastmask : ~0ull;
            const bool own = row >= v.r0 && row < v.r1;
            switch (mode) {
            case HC_THIN:
                base = s & ~(v.hasK ? v.K[gq] : 0ull);
                if (own)
                    v.A[gq] = s;
                break;
            case HC_THICKEN:
                base = ~s & v.A[gq] & valid;
                break;
            case HF_THICKEN:
                base = ~s & valid & ~(v.hasD ? v.Dp[gq] : 0ull);
                if (own)
                    v.A[gq] = s;
                break;
            default:
                base = s & ~v.A[gq];
                break;
            }
        }
        if (__ballot(base != 0) == 0)
            continue;
        uint64_t Vc[I + 1];
        uint32_t E[I + 1];
        {
            uint64_t vm = 0, vc = 0, vp = 0;
            if (base) {
                vm = tile_feat(v, row, w - 1, frame);
                vc = tile_feat(v, row, w, frame);
                vp = tile_feat(v, row, w + 1, frame);
            }
            Vc[0] = vc;
            E[0] = (uint32_t)(vm >> 48) | ((uint32_t)vp << 16);
#pragma unroll
            for (int a = 1; a <= I; ++a) {
                if (base) {
                    vm |= tile_feat(v, row - a, w - 1, frame) | tile_feat(v, row + a, w - 1, frame);
                    vc |= tile_feat(v, row - a, w, frame) | tile_feat(v, row + a, w, frame);
                    vp |= tile_feat(v, row - a, w + 1, frame) | tile_feat(v, row + a, w + 1, frame);
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
                tile_flush(v, cnt, P.rank[k], lrow, w, acc);
                acc = 0;
            }
        }
    }
}

__device__ __forceinline__ void run_tile_stage(int i, const TileView& v, int mode, lds_u32* cnt)
{
    switch (i) {
    case 1: tile_stage<1>(v, mode, cnt); break;
    case 2: tile_stage<2>(v, mode, cnt); break;
    case 3: tile_stage<3>(v, mode, cnt); break;
    case 4: tile_stage<4>(v, mode, cnt); break;
    case 5: tile_stage<5>(v, mode, cnt); break;
    case 6: tile_stage<6>(v, mode, cnt); break;
    case 7: tile_stage<7>(v, mode, cnt); break;
    case 8: tile_stage<8>(v, mode, cnt); break;
    case 9: tile_stage<9>(v, mode, cnt); break;
    case 10: tile_stage<10>(v, mode, cnt); break;
    case 11: tile_stage<11>(v, mode, cnt); break;
    case 12: tile_stage<12>(v, mode, cnt); break;
    case 13: tile_stage<13>(v, mode, cnt); break;
    case 14: tile_stage<14>(v, mode, cnt); break;
    default: tile_stage<15>(v, mode, cnt); break;
    }
}

__device__ int tile_levels_at(int i)
{
    // distinct nonzero sums of two squares <= i^2, i = 0..HASF_R_MAX
    constexpr int tab[HASF_R_MAX + 1] = {
        level_count(0), level_count(1), level_count(2), level_count(3), level_count(4),
        level_count(5), level_count(6), level_count(7), level_count(8), level_count(9),
        level_count(10), level_count(11), level_count(12), level_count(13), level_count(14),
        level_count(15)};
    return tab[i];
}

// The whole band's geometry and planes.
struct Band {
    Img<true> g;
    int t, nt, r0, r1, e0, ER, lo, hi;  // lo, hi: own rows in band coordinates
    int halo;
    size_t SUBG;                        // words per sub-image of an exchange copy
    glb_u32* Xs[2];
};

// Own rows [r0, r0 + halo) and [r1 - halo, r1) (the rows the neighbours
// keep as halo) into exchange copy `out`.
__device__ __forceinline__ void publish(const Band& b, glb_u32* out)
{
    const Img<true>& g = b.g;
    const int WW = g.WW;
    const int top_hi = b.t > 0 ? min(b.r1, b.r0 + b.halo) : b.r0;
    const int bot_lo = b.t < b.nt - 1 ? max(top_hi, b.r1 - b.halo) : b.r1;
    const int ntop = top_hi - b.r0;
    const int n = (ntop + (b.r1 - bot_lo)) * 2 * WW;
    for (int u = threadIdx.x; u < n; u += TILE_NT) {
        const int hr = u / (2 * WW);
        const int rem = u - hr * 2 * WW;
        const int sj = rem >= WW ? 1 : 0;
        const int w = rem - sj * WW;
        const int y = hr < ntop ? b.r0 + hr : bot_lo + (hr - ntop);
        const int si = y & 1;
        out[(size_t)(si * 2 + sj) * b.SUBG + (size_t)(y >> 1) * WW + w] =
            g.S[g.sub(si, sj) + ((y - b.e0) >> 1) * WW + w];
    }
}

// Halo rows [e0, r0) and [r1, e1) from exchange copy `in` (the neighbours'
// own rows). A changed word is written and every word whose test reads it
// (the 3 x 3 word block around it in each sub-image) is flagged; *s_flag
// records that something changed.
__device__ __forceinline__ void refresh_halo(const Band& b, const glb_u32* in, int* s_flag)
{
    const Img<true>& g = b.g;
    const int WW = g.WW;
    const int ntop = b.r0 - b.e0, nbot = b.e0 + b.ER - b.r1;
    const int n = (ntop + nbot) * 2 * WW;
    for (int u = threadIdx.x; u < n; u += TILE_NT) {
        const int hr = u / (2 * WW);
        const int rem = u - hr * 2 * WW;
        const int sj = rem >= WW ? 1 : 0;
        const int w = rem - sj * WW;
        const int y = hr < ntop ? b.e0 + hr : b.r1 + (hr - ntop);
        const int si = y & 1;
        const uint32_t nv = in[(size_t)(si * 2 + sj) * b.SUBG + (size_t)(y >> 1) * WW + w];
        const int rr = (y - b.e0) >> 1;
        const int li = g.sub(si, sj) + rr * WW + w;
        if (g.S[li] != nv) {
            g.S[li] = nv;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int rows_a = (b.ER - a + 1) >> 1;
#pragma unroll
                for (int dr = -1; dr <= 1; ++dr) {
                    const int x = rr + dr;
                    if (x < 0 || x >= rows_a)
                        continue;
#pragma unroll
                    for (int dc = -1; dc <= 1; ++dc) {
                        const int ww = w + dc;
                        if (ww < 0 || ww >= WW)
                            continue;
                        g.D[g.sub(a, 0) + x * WW + ww] = 1;
                        g.D[g.sub(a, 1) + x * WW + ww] = 1;
                    }
                }
            }
            *s_flag = 1;
        }
    }
}

// Levels of one phase in increasing order; in each, epochs of halo / 4
// rounds and one exchange until a round changed nothing anywhere.
__device__ __forceinline__ bool tile_levels(Band& b, const TileView& v, TileSync& ts, int* s_ok, int* s_flag,
                                            lds_u32* cnt, int pi, int nlev, bool thin)
{
    Img<true>& g = b.g;
    Sched sc;
    sched_reset(g, sc);
    __syncthreads();
    for (int k = 0; k < nlev; ++k) {
        if (__hip_atomic_load(&ts.tc->lev[pi][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            continue;  // no tile has a candidate at this level
        const int ser = ++sc.serial;
        ++ts.acts;
        const unsigned c = min(cnt[k], (unsigned)v.slots);
        const size_t eb = (size_t)k * v.slots;
        for (unsigned u = threadIdx.x; u < c; u += TILE_NT) {
            const uint32_t p = v.eidx[eb + u];
            activate_row_word(g, (int)(p >> 10), (int)(p & 1023u), (uint64_t)v.emsk[eb + u], ser);
        }
        __syncthreads();
        const unsigned start = ts.round;
        unsigned lvl_last = start;  // the level's last round that changed something
        for (;;) {
            const int epoch_rounds = b.halo >> 2;
            const int last = run_rounds<true, TILE_NT, true>(g, thin, sc, epoch_rounds, b.lo, b.hi);
            publish(b, b.Xs[ts.gen & 1]);
            // by barrier parity: a tile that reads this epoch's word after
            // the barrier never sees a store of the next epoch (a faster
            // tile can only store the same word again after the barrier
            // that the slower one reaches after reading it)
            unsigned* lcw = &ts.tc->last_change[ts.gen & 1];
            if (last && threadIdx.x == 0)
                __hip_atomic_fetch_max(lcw, ts.round + (unsigned)last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ts.round += (unsigned)epoch_rounds;
            if (!tile_sync(ts, s_ok))
                return false;
            // the last round of the epoch changed no tile's own rows: the
            // level is done (the rounds after its first quiet one were no-ops)
            const unsigned lc = __hip_atomic_load(lcw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool done = lc < ts.round;
            lvl_last = lc > lvl_last ? lc : lvl_last;
            refresh_halo(b, b.Xs[(ts.gen - 1) & 1], s_flag);
            __syncthreads();
            const int f = *s_flag;
            __syncthreads();
            if (f) {
                // as an activation: both copies of the pass serials
                const int hs = ++sc.serial;
                if (threadIdx.x == 0)
                    *s_flag = 0;
                if (threadIdx.x < 4) {
                    g.ctl[CTL_PROD + threadIdx.x] = hs;
                    g.ctl[CTL_PROD2 + threadIdx.x] = hs;
                }
            }
            if (done) {
                ts.rounds += (lvl_last - start) + 1u;
                break;
            }
        }
    }
    return true;
}

__device__ __forceinline__ bool tile_image(const ImgDesc* __restrict__ dp, TileSync& ts, int* s_ok, int* s_flag,
                                           uint64_t* smem, lds_u32* cnt, lds_i32* ctl, int TH, int ERmax, int halo)
{
    const int H = dp->H, W = dp->W;
    Band b;
    b.halo = halo;
    b.t = blockIdx.x;
    b.nt = gridDim.x;
    b.r0 = b.t * TH;
    b.r1 = min(H, b.r0 + TH);
    b.e0 = max(0, b.r0 - halo);
    b.ER = min(H, b.r1 + halo) - b.e0;
    b.lo = b.r0 - b.e0;
    b.hi = b.r1 - b.e0;
    Img<true>& g = b.g;
    g.ctl = ctl;
    g.H = b.ER;
    g.W = W;
    bind_state(g, (void*)smem);
    g.A = g.K = g.Dp = nullptr;
    g.eidx = nullptr;
    g.emsk = nullptr;
    g.hasK = dp->C != nullptr;
    g.hasD = dp->D != nullptr;
    g.conn4 = dp->conn4 != 0;
    const int WW = g.WW;
    const size_t NWD = (size_t)H * WW;
    glb_u64* Rg = (glb_u64*)dp->gplanes;
    glb_u64* A = Rg + NWD;
    glb_u64* K = A + NWD;
    glb_u64* Dp = K + NWD;
    const size_t xs_words = hasf_align256(tile_sub_words(H, W) * 4) / 4;
    b.SUBG = tile_sub_words(H, W) / 4;
    b.Xs[0] = (glb_u32*)((glb_u8*)dp->gplanes + hasf_align256(4 * NWD * 8));
    b.Xs[1] = b.Xs[0] + xs_words;
    const int r = dp->r;
    const int nlev_max = r > 0 ? tile_levels_at(r) : 1;
    TileView v;
    v.Rg = Rg;
    v.A = A;
    v.K = K;
    v.Dp = Dp;
    v.slots = (size_t)ERmax * WW;
    v.eidx = (glb_u32*)dp->ent_idx + (size_t)b.t * nlev_max * v.slots;
    v.emsk = (glb_u64*)dp->ent_msk + (size_t)b.t * nlev_max * v.slots;
    v.H = H;
    v.WW = WW;
    v.lastmask = g.lastmask;
    v.e0 = b.e0;
    v.ER = b.ER;
    v.r0 = b.r0;
    v.r1 = b.r1;
    v.hasK = g.hasK;
    v.hasD = g.hasD;
    const int tid = threadIdx.x;
    const long long ld = dp->ld;

    // own rows packed into the global planes, then the band into LDS
    pack_rows(dp->X + (long long)b.r0 * ld, dp->C ? dp->C + (long long)b.r0 * ld : nullptr, ld, b.r1 - b.r0, W,
              Rg + (size_t)b.r0 * WW, g.hasK ? K + (size_t)b.r0 * WW : nullptr, tid, TILE_NT);
    if (g.hasD)
        pack_background(dp->D + (long long)b.r0 * ld, ld, b.r1 - b.r0, W, Rg + (size_t)b.r0 * WW,
                        Dp + (size_t)b.r0 * WW, tid, TILE_NT);
    if (!tile_sync(ts, s_ok))
        return false;
    for (int q = tid; q < b.ER * WW; q += TILE_NT)
        g.R[q] = Rg[(size_t)b.e0 * WW + q];
    __syncthreads();
    rows_to_sub(g, tid, TILE_NT);
    __syncthreads();

    const int rot = dp->order ? 2 : 0;  // as in the per-image kernel
    int pi = 0;
    for (int i = 1; i <= r; ++i) {
        const int nlev = tile_levels_at(i);
        for (int k = 0; k < 4; ++k, ++pi) {
            const int ph = (k + rot) & 3;
            if (pi > 0) {
                // own rows of the set into the row-major copy the stages read
                for (int q = b.lo * WW + tid; q < b.hi * WW; q += TILE_NT) {
                    const int lr = q / WW;
                    const int w = q - lr * WW;
                    const int o = (lr >> 1) * WW + w;
                    Rg[(size_t)b.e0 * WW + q] =
                        spread_bits(g.S[g.sub(lr & 1, 0) + o]) | (spread_bits(g.S[g.sub(lr & 1, 1) + o]) << 1);
                }
                if (!tile_sync(ts, s_ok))
                    return false;
            }
            clear_candidates(g, tid, TILE_NT);
            for (int q = tid; q < nlev; q += TILE_NT)
                cnt[q] = 0;
            __syncthreads();
            run_tile_stage(i, v, ph, cnt);
            __syncthreads();
            for (int q = tid; q < nlev; q += TILE_NT)
                if (cnt[q])
                    __hip_atomic_store(&ts.tc->lev[pi][q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!tile_sync(ts, s_ok))
                return false;
            if (!tile_levels(b, v, ts, s_ok, s_flag, cnt, pi, nlev, ph == HC_THIN || ph == HF_THIN))
                return false;
        }
    }
    // the own rows of the result
    sub_to_rows(g, tid, TILE_NT);
    __syncthreads();
    unpack_rows(dp->X + (long long)b.r0 * ld, ld, b.r1 - b.r0, W, g.R + (size_t)b.lo * WW, tid, TILE_NT);
    return true;
}

}  // namespace

// One image over gridDim.x row tiles of TH own rows and `halo` halo rows
// (ERmax: the longest band, which sizes the entry lists). If a grid barrier
// gave up, tc->err and the caller's sticky word are set (the image is then
// undefined).
__global__ __launch_bounds__(TILE_NT) void hasf_tile_kernel(const ImgDesc* __restrict__ dp, TileCtl* tc,
                                                            unsigned* err_out, int TH, int ERmax, int halo)
{
    extern __shared__ uint64_t smem[];
    __shared__ unsigned cnt[HASF_LEVELS_MAX];
    __shared__ int ctl[CTL_LDS_WORDS];
    __shared__ int s_ok, s_flag;
    if (threadIdx.x == 0)
        s_flag = 0;
    TileSync ts{tc, gridDim.x, 0u, 0u, 0u, 0u};
    const bool ok = tile_image(dp, ts, &s_ok, &s_flag, smem, (lds_u32*)cnt, (lds_i32*)ctl, TH, ERmax, halo);
    if (!ok && threadIdx.x == 0) {
        __hip_atomic_store(&tc->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (err_out)
            __hip_atomic_fetch_or(err_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (ok && err_out && blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned long long* c = reinterpret_cast<unsigned long long*>(err_out + GRID_COUNTS_OFF);
        __hip_atomic_fetch_add(c + 0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 1, (unsigned long long)ts.rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 2, (unsigned long long)ts.acts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(c + 3, (unsigned long long)ts.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

namespace hasf_detail {

hipError_t launch_tile(const ImgDesc* d_desc, TileCtl* d_ctl, unsigned* d_err, const TilePlan& P,
                       hipStream_t stream)
{
    static std::atomic<uint64_t> attr{0};
    const hipError_t e = allow_dyn_lds((const void*)hasf_tile_kernel, 160 * 1024 - 2048, attr);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(hasf_tile_kernel, dim3(P.ntiles), dim3(TILE_NT), P.lds_bytes, stream, d_desc, d_ctl, d_err,
                       P.TH, P.ER, P.halo);
    return hipGetLastError();
}

}  // namespace hasf_detail
