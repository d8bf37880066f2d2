// One large image filtered by tiles whose state stays in LDS (the schedule
// of thinning H and thickening *H of Sec. 2, run with temporal blocking).
//
// The image is cut into row bands of TH rows, and each band into column
// tiles of whole 64-column words. Tile t (one workgroup) owns rows [r0, r1)
// and words [cw0, cw1) of its band and also keeps `halo` rows above and below
// and TILE_HALO_WORDS words left and right that its neighbours own, so its
// LDS state is a block of up to TH + 2 halo rows in the layout of the
// per-image kernel. A subfield pass decides a pixel from its 3x3
// neighbourhood, so after k passes a block can differ from the whole-image
// schedule only within k rows or columns of its cut edges: a tile runs
// halo / 4 rounds (4 passes each, halo passes in all, at most 16 < 64
// columns) on its own and its own pixels are then exactly the schedule's.
// Then every tile publishes its own pixels that its neighbours keep (its
// first and last halo rows, its first and last halo words), the tiles meet at
// one grid barrier, and each replaces its halo with its neighbours' pixels
// (flagging every word whose test reads a changed word). A level of the schedule ends after the first round that
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
#include <algorithm>
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
    unsigned rounds;  // rounds of the schedule (wave 0 of workgroup 0)
    unsigned acts;    // levels activated (uniform)
    unsigned cchg;    // high half of the barrier word last seen (thread 0)
};

// Grid barrier. Every wave first waits until its own stores have completed;
// then one thread per workgroup counts the workgroup in and waits for the
// last arrival to publish the new generation. Bounded: on time-out, or when
// another workgroup gave up, it returns false.
//
// `fenced` (the barriers around the distance stages): a device-scope release
// before the arrival and an acquire after it, so that the plain stores of the
// row-major planes are visible to every later plain load. The epoch barriers
// go without them: the only data that crosses them, the exchange copies, is
// written and read with device-scope atomic stores and loads, which are
// coherent across the XCDs' L2 caches by themselves, and a store counts as
// complete for the wait only once it is visible at that scope. Skipping the
// fences keeps each L2's lines (level entries, planes) valid and spares the
// write-back of its dirty lines at every epoch.
//
// `chg` (uniform): this tile's last round changed one of its own rows. Such
// arrivals are counted in the high half of the arrival word, and the last
// arrival copies the running count into the barrier word, so each tile
// learns without another memory round trip whether any tile did: *s_quiet
// is 1 when none did.
__device__ __forceinline__ bool tile_sync(TileSync& ts, int* s_ok, bool fenced, bool chg = false,
                                          int* s_quiet = nullptr)
{
    __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
        TileCtl* tc = ts.tc;
        int ok = 1;
        if (fenced)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long add = 1ull | ((unsigned long long)(chg ? 1u : 0u) << 32);
        const unsigned long long old =
            __hip_atomic_fetch_add(&tc->bar_arrive, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long word;
        if ((unsigned)old + 1u == (ts.gen + 1) * ts.nblk) {
            word = (unsigned long long)(ts.gen + 1) | ((old + add) & 0xFFFFFFFF00000000ull);
            __hip_atomic_store(&tc->bar_word, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            for (unsigned it = 1;; ++it) {
                word = __hip_atomic_load(&tc->bar_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)word != ts.gen)
                    break;
                // the abort word and the clock only now and then: one load
                // per poll keeps the release latency down
                if ((it & 31u) == 0) {
                    if (__hip_atomic_load(&tc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        ok = 0;
                        break;
                    }
                    if (wall_clock64() - t0 > TILE_WAIT_LIMIT) {
                        __hip_atomic_store(&tc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (fenced)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const unsigned cum = (unsigned)(word >> 32);
        if (s_quiet)
            *s_quiet = cum == ts.cchg ? 1 : 0;
        ts.cchg = cum;
        *s_ok = ok;
    }
    ++ts.gen;
    __syncthreads();
    return *s_ok != 0;
}

// The exchange copies cross the unfenced epoch barriers: device-scope atomic
// stores and loads only.
__device__ __forceinline__ void xs_store(glb_u32* p, uint32_t v)
{
    __hip_atomic_store((uint32_t*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t xs_load(const glb_u32* p)
{
    return __hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    int e0, ER, r0, r1;  // block rows [e0, e0 + ER); own rows [r0, r1)
    int bw0, WWb, cw0, cw1;  // block words [bw0, bw0 + WWb); own words [cw0, cw1)
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
    const int nwb = v.ER * v.WWb;
    const int nq = (nwb + TILE_NT - 1) / TILE_NT * TILE_NT;
    for (int q = threadIdx.x; q < nq; q += TILE_NT) {
        uint64_t base = 0;
        int lrow = 0, wb = 0, w = 0, row = 0;
        if (q < nwb) {
            lrow = q / v.WWb;
            wb = q - lrow * v.WWb;
            w = v.bw0 + wb;  // image word
            row = v.e0 + lrow;
            const size_t gq = (size_t)row * v.WW + w;
            const uint64_t s = v.Rg[gq];
            const uint64_t valid = (w == v.WW - 1) ? v.lastmask : ~0ull;
            const bool own = row >= v.r0 && row < v.r1 && w >= v.cw0 && w < v.cw1;
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
                tile_flush(v, cnt, P.rank[k], lrow, wb, acc);
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
    int tr, nr, tc, nc;                 // row band and column tile, and their counts
    int r0, r1, e0, ER, lo, hi;         // lo, hi: own rows in block coordinates
    int cw0, cw1, bw0, WWg;             // own words, first block word, words of an image row
    int halo;
    size_t SUBG;                        // words per sub-image of an exchange copy
    glb_u32* Xs[2];
};

// The own pixels the neighbours keep as halo, into exchange copy `out`
// (image coordinates): own rows [r0, r0 + halo) and [r1 - halo, r1) over the
// own words, and the own words [cw0, cw0 + hw) and [cw1 - hw, cw1) over the
// own rows (hw = TILE_HALO_WORDS; only towards existing neighbours).
__device__ __forceinline__ void publish(const Band& b, glb_u32* out)
{
    const Img<true>& g = b.g;
    const int WWb = g.WW, nw = b.cw1 - b.cw0;
    const int top_hi = b.tr > 0 ? min(b.r1, b.r0 + b.halo) : b.r0;
    const int bot_lo = b.tr < b.nr - 1 ? max(top_hi, b.r1 - b.halo) : b.r1;
    const int ntop = top_hi - b.r0;
    auto put = [&](int y, int gw, int sj) {
        const int si = y & 1;
        xs_store(out + (size_t)(si * 2 + sj) * b.SUBG + (size_t)(y >> 1) * b.WWg + gw,
                 g.S[g.sub(si, sj) + ((y - b.e0) >> 1) * WWb + (gw - b.bw0)]);
    };
    const int n = (ntop + (b.r1 - bot_lo)) * 2 * nw;
    for (int u = threadIdx.x; u < n; u += TILE_NT) {
        const int hr = u / (2 * nw);
        const int rem = u - hr * 2 * nw;
        const int sj = rem >= nw ? 1 : 0;
        const int w = rem - sj * nw;
        put(hr < ntop ? b.r0 + hr : bot_lo + (hr - ntop), b.cw0 + w, sj);
    }
    // edge words of the own rows (the rows above are published twice when
    // they are also in the first and last halo rows: the same value)
    const int hl = b.tc > 0 ? min(TILE_HALO_WORDS, nw) : 0;
    const int hrr = b.tc < b.nc - 1 ? min(TILE_HALO_WORDS, nw) : 0;
    const int ne = hl + hrr;
    if (ne == 0)
        return;
    const int m = (b.r1 - b.r0) * 2 * ne;
    for (int u = threadIdx.x; u < m; u += TILE_NT) {
        const int y = b.r0 + u / (2 * ne);
        const int rem = u % (2 * ne);
        const int sj = rem >= ne ? 1 : 0;
        const int k = rem - sj * ne;
        put(y, k < hl ? b.cw0 + k : b.cw1 - hrr + (k - hl), sj);
    }
}

// The halo from exchange copy `in` (the neighbours' own pixels): rows
// [e0, r0) and [r1, e1) over all block words, and the halo words left and
// right of the own words over the own rows. A changed word is written and
// every word whose test reads it (the 3 x 3 word block around it in each
// sub-image) is flagged; *s_flag records that something changed.
__device__ __forceinline__ void refresh_halo(const Band& b, const glb_u32* in, int* s_flag)
{
    const Img<true>& g = b.g;
    const int WWb = g.WW;
    const int ntop = b.r0 - b.e0, nbot = b.e0 + b.ER - b.r1;
    const int n = (ntop + nbot) * 2 * WWb;  // halo rows over the block words
    const int hl = b.cw0 - b.bw0, hrr = b.bw0 + WWb - b.cw1;
    const int ne = hl + hrr;
    const int m = (b.r1 - b.r0) * 2 * ne;  // halo words over the own rows
    // item u: its image row y, block word wb and column parity sj
    auto item = [&](int u, int& y, int& wb, int& sj) {
        if (u < n) {
            const int hr = u / (2 * WWb);
            const int rem = u - hr * 2 * WWb;
            sj = rem >= WWb ? 1 : 0;
            wb = rem - sj * WWb;
            y = hr < ntop ? b.e0 + hr : b.r1 + (hr - ntop);
        } else {
            u -= n;  // here ne > 0
            y = b.r0 + u / (2 * ne);
            const int rem = u % (2 * ne);
            sj = rem >= ne ? 1 : 0;
            const int k = rem - sj * ne;
            wb = k < hl ? k : (b.cw1 - b.bw0) + (k - hl);
        }
    };
    auto put = [&](int y, int wb, int sj, uint32_t nv) {
        const int si = y & 1;
        const int rr = (y - b.e0) >> 1;
        const int li = g.sub(si, sj) + rr * WWb + wb;
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
                        const int ww = wb + dc;
                        if (ww < 0 || ww >= WWb)
                            continue;
                        g.D[g.sub(a, 0) + x * WWb + ww] = 1;
                        g.D[g.sub(a, 1) + x * WWb + ww] = 1;
                    }
                }
            }
            *s_flag = 1;
        }
    };
    // K items per thread and batch: their loads are all in flight before
    // the first is compared, one memory round trip per batch
    constexpr int K = 2;
    const int T = n + m;
    for (int base = 0; base < T; base += K * TILE_NT) {
        uint32_t nv[K];
        int yy[K], ww[K], ss[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int u = base + k * TILE_NT + (int)threadIdx.x;
            yy[k] = -1;
            ww[k] = ss[k] = 0;
            nv[k] = 0;
            if (u < T) {
                item(u, yy[k], ww[k], ss[k]);
                nv[k] = xs_load(in + (size_t)((yy[k] & 1) * 2 + ss[k]) * b.SUBG + (size_t)(yy[k] >> 1) * b.WWg +
                                (b.bw0 + ww[k]));
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (yy[k] >= 0)
                put(yy[k], ww[k], ss[k], nv[k]);
    }
}

// Levels of one phase in increasing order; in each, epochs of halo / 4
// rounds and one exchange until a round changed nothing anywhere.
__device__ __forceinline__ bool tile_levels(Band& b, const TileView& v, TileSync& ts, int* s_ok, int* s_flag,
                                            int* s_quiet, lds_u32* cnt, lds_u32* levf, int pi, int nlev, bool thin)
{
    Img<true>& g = b.g;
    Sched sc;
    sched_reset(g, sc);
    // which levels some tile has candidates at (set before the last barrier)
    for (int q = threadIdx.x; q < nlev; q += TILE_NT)
        levf[q] = __hip_atomic_load(&ts.tc->lev[pi][q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // the round statistics: all of wave 0 of workgroup 0 (a wave-uniform branch,
    // so the load of the change word is not waited for where it is issued)
    const bool stats = blockIdx.x == 0 && threadIdx.x < 64;
    const int epoch_rounds = b.halo >> 2;
    // the next level after k that some tile has candidates at (uniform)
    auto next_level = [&](int k) {
        int kn = k + 1;
        while (kn < nlev && levf[kn] == 0)
            ++kn;
        return __builtin_amdgcn_readfirstlane(kn);
    };
    auto entries = [&](int k) {
        return k < nlev ? (unsigned)__builtin_amdgcn_readfirstlane((int)min(cnt[k], (unsigned)v.slots)) : 0u;
    };
    // marks level k's candidates of this tile live; the first entry of each
    // thread may come in registers (have)
    auto activate = [&](int k, unsigned c, bool have, uint32_t pi0, uint64_t pm0) {
        const int ser = ++sc.serial;
        ++ts.acts;
        const size_t eb = (size_t)k * v.slots;
        for (unsigned u = threadIdx.x; u < c; u += TILE_NT) {
            uint32_t p = pi0;
            uint64_t m = pm0;
            if (!have || u >= TILE_NT) {
                p = v.eidx[eb + u];
                m = (uint64_t)v.emsk[eb + u];
            }
            activate_row_word(g, (int)(p >> 10), (int)(p & 1023u), m, ser);
        }
        __syncthreads();
    };
    int k = next_level(-1);
    if (k >= nlev)
        return true;
    activate(k, entries(k), false, 0u, 0ull);
    int kn = next_level(k);
    unsigned cn = entries(kn);
    unsigned start = ts.round;
    unsigned lvl_last = start;  // the level's last round that changed something (statistics)
    for (;;) {
        const int last = run_rounds<true, TILE_NT, true>(g, thin, sc, epoch_rounds, b.lo, b.hi, b.cw0 - b.bw0,
                                                         b.cw1 - b.bw0);
        publish(b, b.Xs[ts.gen & 1]);
        // for the round count only, by barrier parity: workgroup 0 reads
        // this epoch's word after the barrier and before it arrives at the
        // next one, which no tile passes before it arrives, so no store of
        // the epoch after the next can have reached the word
        unsigned* lcw = &ts.tc->last_change[ts.gen & 1];
        if (last && threadIdx.x == 0)
            __hip_atomic_fetch_max(lcw, ts.round + (unsigned)last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ts.round += (unsigned)epoch_rounds;
        if (!tile_sync(ts, s_ok, false, last == epoch_rounds, s_quiet))
            return false;
        // the last round of the epoch changed no tile's own rows: the level
        // is done (the rounds after its first quiet one were no-ops)
        const bool done = *s_quiet != 0;
        unsigned lc = 0;
        if (stats)
            lc = __hip_atomic_load(lcw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the next level's first entries, loaded with the halo: both are in
        // flight together, so its activation waits for no load of its own
        uint32_t pi0 = 0;
        uint64_t pm0 = 0;
        if (done && threadIdx.x < cn) {
            pi0 = v.eidx[(size_t)kn * v.slots + threadIdx.x];
            pm0 = (uint64_t)v.emsk[(size_t)kn * v.slots + threadIdx.x];
        }
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
        // (the empty asm keeps the compiler from moving this maximum, and with
        // it the wait for lc, up to the load)
        asm volatile("" : "+v"(lc));
        lvl_last = lc > lvl_last ? lc : lvl_last;
        if (done) {
            ts.rounds += (lvl_last - start) + 1u;
            if (kn >= nlev)
                break;
            activate(kn, cn, true, pi0, pm0);
            k = kn;
            kn = next_level(k);
            cn = entries(kn);
            start = ts.round;
            lvl_last = start;
        }
    }
    return true;
}

__device__ __forceinline__ bool tile_image(const ImgDesc* __restrict__ dp, TileSync& ts, int* s_ok, int* s_flag,
                                           int* s_quiet, uint64_t* smem, lds_u32* cnt, lds_u32* levf, lds_i32* ctl, int TH, int ERmax, int halo,
                                           int nc, int WWbmax, int nxcd)
{
    const int H = dp->H, W = dp->W;
    const int WW = (W + 63) >> 6;
    Band b;
    b.halo = halo;
    // tiles of one XCD form a run (workgroups are dealt to the XCDs round
    // robin), so most halo exchanges stay within one L2
    const int nx = nxcd > 1 && gridDim.x % nxcd == 0 ? nxcd : 1;
    const int t = (int)(blockIdx.x % nx) * (int)(gridDim.x / nx) + (int)(blockIdx.x / nx);
    b.nc = nc;
    b.nr = (int)gridDim.x / nc;
    b.tr = t / nc;
    b.tc = t - b.tr * nc;
    b.r0 = b.tr * TH;
    b.r1 = min(H, b.r0 + TH);
    b.e0 = max(0, b.r0 - halo);
    b.ER = min(H, b.r1 + halo) - b.e0;
    b.lo = b.r0 - b.e0;
    b.hi = b.r1 - b.e0;
    b.WWg = WW;
    b.cw0 = tile_cw0(b.tc, nc, WW);
    b.cw1 = tile_cw0(b.tc + 1, nc, WW);
    b.bw0 = nc > 1 ? max(0, b.cw0 - TILE_HALO_WORDS) : 0;
    const int bw1 = nc > 1 ? min(WW, b.cw1 + TILE_HALO_WORDS) : WW;
    Img<true>& g = b.g;
    g.ctl = ctl;
    g.H = b.ER;
    // the block's columns: whole words, up to the image's last column
    g.W = min(W, 64 * bw1) - 64 * b.bw0;
    bind_state(g, (void*)smem);
    g.A = g.K = g.Dp = nullptr;
    g.eidx = nullptr;
    g.emsk = nullptr;
    g.hasK = dp->C != nullptr;
    g.hasD = dp->D != nullptr;
    g.conn4 = dp->conn4 != 0;
    const int WWb = g.WW;  // bw1 - bw0
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
    v.slots = (size_t)ERmax * WWbmax;
    v.eidx = (glb_u32*)dp->ent_idx + (size_t)t * nlev_max * v.slots;
    v.emsk = (glb_u64*)dp->ent_msk + (size_t)t * nlev_max * v.slots;
    v.H = H;
    v.WW = WW;
    v.lastmask = (W & 63) ? ((1ull << (W & 63)) - 1ull) : ~0ull;
    v.e0 = b.e0;
    v.ER = b.ER;
    v.r0 = b.r0;
    v.r1 = b.r1;
    v.bw0 = b.bw0;
    v.WWb = WWb;
    v.cw0 = b.cw0;
    v.cw1 = b.cw1;
    v.hasK = g.hasK;
    v.hasD = g.hasD;
    const int tid = threadIdx.x;
    const long long ld = dp->ld;
    const int nown = b.cw1 - b.cw0;
    const int own_lo = b.cw0 - b.bw0;  // first own word in the block

    // own pixels packed into the global planes, then the block into LDS
    const bool vec_ok = ((((uintptr_t)dp->X) | (dp->C ? (uintptr_t)dp->C : 0) |
                          (dp->D ? (uintptr_t)dp->D : 0) | (uintptr_t)ld) & 15) == 0;
    for (int q = tid; q < (b.r1 - b.r0) * nown; q += TILE_NT) {
        const int row = b.r0 + q / nown;
        const int w = b.cw0 + q % nown;
        const int n = min(64, W - 64 * w);
        const size_t gq = (size_t)row * WW + w;
        const uint64_t m = pack_word(dp->X + (long long)row * ld + 64 * w, n, vec_ok);
        Rg[gq] = m;
        if (g.hasK)
            K[gq] = pack_word(dp->C + (long long)row * ld + 64 * w, n, vec_ok) & m;
        if (g.hasD)
            Dp[gq] = pack_word(dp->D + (long long)row * ld + 64 * w, n, vec_ok) & ~m;
    }
    if (!tile_sync(ts, s_ok, true))
        return false;
    for (int q = tid; q < b.ER * WWb; q += TILE_NT) {
        const int lr = q / WWb;
        g.R[q] = Rg[(size_t)(b.e0 + lr) * WW + b.bw0 + (q - lr * WWb)];
    }
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
                // own pixels of the set into the row-major copy the stages read
                for (int q = tid; q < (b.hi - b.lo) * nown; q += TILE_NT) {
                    const int lr = b.lo + q / nown;
                    const int wb = own_lo + q % nown;
                    const int o = (lr >> 1) * WWb + wb;
                    Rg[(size_t)(b.e0 + lr) * WW + b.bw0 + wb] =
                        spread_bits(g.S[g.sub(lr & 1, 0) + o]) | (spread_bits(g.S[g.sub(lr & 1, 1) + o]) << 1);
                }
                if (!tile_sync(ts, s_ok, true))
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
            if (!tile_sync(ts, s_ok, true))
                return false;
            if (!tile_levels(b, v, ts, s_ok, s_flag, s_quiet, cnt, levf, pi, nlev, ph == HC_THIN || ph == HF_THIN))
                return false;
        }
    }
    // the own pixels of the result
    sub_to_rows(g, tid, TILE_NT);
    __syncthreads();
    for (int q = tid; q < (b.r1 - b.r0) * nown; q += TILE_NT) {
        const int lr = b.lo + q / nown;
        const int wb = own_lo + q % nown;
        const int w = b.bw0 + wb;
        unpack_word(dp->X + (long long)(b.e0 + lr) * ld + 64 * w, min(64, W - 64 * w), g.R[lr * WWb + wb],
                    vec_ok);
    }
    return true;
}

}  // namespace

// One image over gridDim.x tiles: nc column tiles per band of TH own rows,
// `halo` halo rows (ERmax rows and WWbmax words: the largest block, which
// sizes the entry lists). If a grid barrier
// gave up, tc->err and the caller's sticky word are set (the image is then
// undefined).
__global__ __launch_bounds__(TILE_NT) void hasf_tile_kernel(const ImgDesc* __restrict__ dp, TileCtl* tc,
                                                            unsigned* err_out, int TH, int ERmax, int halo, int nc,
                                                            int WWbmax, int nxcd)
{
    extern __shared__ uint64_t smem[];
    __shared__ unsigned cnt[HASF_LEVELS_MAX];
    __shared__ unsigned levf[HASF_LEVELS_MAX];
    __shared__ int ctl[CTL_LDS_WORDS];
    __shared__ int s_ok, s_flag, s_quiet;
    if (threadIdx.x == 0)
        s_flag = 0;
    TileSync ts{tc, gridDim.x, 0u, 0u, 0u, 0u, 0u};
    const bool ok = tile_image(dp, ts, &s_ok, &s_flag, &s_quiet, smem, (lds_u32*)cnt, (lds_u32*)levf, (lds_i32*)ctl,
                               TH, ERmax, halo, nc, WWbmax, nxcd);
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

hipError_t launch_tile(const ImgDesc* d_desc, TileCtl* d_ctl, unsigned* d_err, const TilePlan& P, int nxcd,
                       hipStream_t stream)
{
    static std::atomic<uint64_t> attr{0};
    const hipError_t e = allow_dyn_lds((const void*)hasf_tile_kernel, 160 * 1024 - 2048, attr);
    if (e != hipSuccess)
        return e;
    // more than half a CU's LDS: one tile per CU (at most one tile per CU
    // is planned), so that the dispatcher cannot put two tiles on one CU
    // while others stay idle
    const size_t lds = std::max(P.lds_bytes, (size_t)(80 * 1024 + 256));
    hipLaunchKernelGGL(hasf_tile_kernel, dim3(P.ntiles), dim3(TILE_NT), lds, stream, d_desc, d_ctl, d_err, P.TH,
                       P.ER, P.halo, P.nc, P.WWb, nxcd);
    return hipGetLastError();
}

}  // namespace hasf_detail
