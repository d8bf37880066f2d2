// Device code shared by the libhasf kernels: bit-packed planes, packing of
// byte images, and the subfield rounds of thinning / thickening.
#pragma once

#include <type_traits>

#include "hasf_common.h"

namespace hasf_dev {

constexpr int BLOCK = 512;
constexpr uint64_t EVEN_COLS = 0x5555555555555555ull;
constexpr uint64_t ODD_COLS = 0xAAAAAAAAAAAAAAAAull;

// explicit address spaces keep LDS accesses on ds_* and global ones on
// global_* instructions across non-inlined calls
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(1))) uint64_t glb_u64;
typedef __attribute__((address_space(1))) uint32_t glb_u32;
typedef __attribute__((address_space(3))) unsigned lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(1))) uint8_t glb_u8;

enum StageMode {
    HC_THIN = 0,     // features = complement u outside; base = S \ K; saves S into A
    HC_THICKEN = 1,  // features = S; base = A \ S
    HF_THICKEN = 2,  // features = S; base = window \ S; saves S into A
    HF_THIN = 3      // features = complement u outside; base = S \ A
};

template <bool LDS>
struct Img {
    using P = typename std::conditional<LDS, lds_u64*, glb_u64*>::type;
    using PD = typename std::conditional<LDS, lds_u8*, glb_u8*>::type;
    P S;          // current set
    P M;          // activated candidates of the running phase
    PD D0, D1;    // per word: must be re-tested in the even / odd column subfield
    glb_u64* A;   // set saved before the phase
    glb_u64* K;   // constraint set
    glb_u32* eidx;
    glb_u64* emsk;
    int H, W, WW, NWD;
    int E;              // first word of the odd-row half of a plane
    uint64_t lastmask;  // valid bits of the last word of a row
    bool hasK;

    // Planes are stored split by row parity: the even rows first, then the odd
    // rows, so that the words of one subfield pass and of its neighbouring
    // rows are contiguous in memory (conflict-free LDS access per wave).
    __device__ __forceinline__ int at(int row, int w) const
    {
        return ((row & 1) ? E : 0) + (row >> 1) * WW + w;
    }
    // row and word of memory index q
    __device__ __forceinline__ void rowcol(int q, int& row, int& w) const
    {
        const bool odd = q >= E;
        const int r2 = odd ? q - E : q;
        const int rr = r2 / WW;
        w = r2 - rr * WW;
        row = 2 * rr + (odd ? 1 : 0);
    }
};

template <bool LDS>
__device__ __forceinline__ Img<LDS> make_img(const ImgDesc* __restrict__ dp, uint64_t* smem)
{
    Img<LDS> g;
    g.H = dp->H;
    g.W = dp->W;
    g.WW = (g.W + 63) >> 6;
    g.NWD = g.H * g.WW;
    g.E = ((g.H + 1) >> 1) * g.WW;
    g.lastmask = (g.W & 63) ? ((1ull << (g.W & 63)) - 1ull) : ~0ull;
    glb_u64* gp = (glb_u64*)dp->gplanes;
    if constexpr (LDS) {
        g.S = (lds_u64*)smem;
        g.M = (lds_u64*)smem + g.NWD;
        g.D0 = (lds_u8*)((lds_u64*)smem + 2 * (size_t)g.NWD);
        g.D1 = g.D0 + g.NWD;
        g.A = gp;
        g.K = gp + g.NWD;
    } else {
        g.S = gp;
        g.M = gp + g.NWD;
        g.A = gp + 2 * (size_t)g.NWD;
        g.K = gp + 3 * (size_t)g.NWD;
        g.D0 = (glb_u8*)(gp + 4 * (size_t)g.NWD);
        g.D1 = g.D0 + g.NWD;
    }
    g.hasK = dp->C != nullptr;
    g.eidx = (glb_u32*)dp->ent_idx;
    g.emsk = (glb_u64*)dp->ent_msk;
    return g;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// 4 bytes -> 4 bits (bit k = byte k nonzero)
__device__ __forceinline__ uint32_t nz4(uint32_t v)
{
    uint32_t t = v | (v >> 4);
    t |= t >> 2;
    t |= t >> 1;
    t &= 0x01010101u;
    return ((t * 0x00204081u) >> 21) & 0xFu;
}

// 4 bits -> 4 bytes of 0/1
__device__ __forceinline__ uint32_t expand4(uint32_t nib)
{
    return (nib * 0x00204081u) & 0x01010101u;
}

// Pack nonzero bytes of X (and C) into words: one thread per word.
template <bool LDS>
__device__ void pack_image(const uint8_t* __restrict__ X, const uint8_t* __restrict__ C, long long ld,
                           const Img<LDS>& g)
{
    const bool vec_ok = ((((uintptr_t)X) | (C ? (uintptr_t)C : 0) | (uintptr_t)ld) & 15) == 0;
    for (int q = threadIdx.x; q < g.NWD; q += BLOCK) {
        int row, w;
        g.rowcol(q, row, w);
        const int c0 = w * 64;
        const uint8_t* xr = X + (long long)row * ld + c0;
        const uint8_t* cr = C ? C + (long long)row * ld + c0 : nullptr;
        uint64_t m = 0, k = 0;
        if (vec_ok && c0 + 64 <= g.W) {
            const uint4* xp = reinterpret_cast<const uint4*>(xr);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint4 v = xp[j];
                uint64_t bits = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
                m |= bits << (16 * j);
            }
            if (cr) {
                const uint4* cp = reinterpret_cast<const uint4*>(cr);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint4 v = cp[j];
                    uint64_t bits = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
                    k |= bits << (16 * j);
                }
            }
        } else {
            const int n = min(64, g.W - c0);
            for (int j = 0; j < n; ++j) {
                m |= (uint64_t)(xr[j] != 0) << j;
                if (cr)
                    k |= (uint64_t)(cr[j] != 0) << j;
            }
        }
        g.S[q] = m;
        if (g.hasK)
            g.K[q] = k & m;
    }
}

template <bool LDS>
__device__ void unpack_image(uint8_t* __restrict__ X, long long ld, const Img<LDS>& g)
{
    const bool vec_ok = ((((uintptr_t)X) | (uintptr_t)ld) & 15) == 0;
    for (int q = threadIdx.x; q < g.NWD; q += BLOCK) {
        int row, w;
        g.rowcol(q, row, w);
        const int c0 = w * 64;
        uint8_t* xr = X + (long long)row * ld + c0;
        const uint64_t m = g.S[q];
        if (vec_ok && c0 + 64 <= g.W) {
            uint4* xp = reinterpret_cast<uint4*>(xr);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t b16 = (uint32_t)(m >> (16 * j)) & 0xFFFFu;
                uint4 v;
                v.x = expand4(b16 & 0xF);
                v.y = expand4((b16 >> 4) & 0xF);
                v.z = expand4((b16 >> 8) & 0xF);
                v.w = expand4((b16 >> 12) & 0xF);
                xp[j] = v;
            }
        } else {
            const int n = min(64, g.W - c0);
            for (int j = 0; j < n; ++j)
                xr[j] = (uint8_t)((m >> j) & 1u);
        }
    }
}

// word (row, w) of a plane, 0 outside the window
template <bool LDS, typename PP>
__device__ __forceinline__ uint64_t ld_word(const Img<LDS>& g, PP p, int row, int w)
{
    if (row < 0 || row >= g.H || w < 0 || w >= g.WW)
        return 0;
    return p[g.at(row, w)];
}

// Rounds of the four subfield passes (even,even) (even,odd) (odd,even)
// (odd,odd) until a round changes nothing. A pass tests, on the state left by
// the previous pass, the activated candidates of its subfield and flips the
// simple ones (thinning deletes, thickening adds). Two points of one subfield
// are never 8-adjacent, so a pass is a pure data-parallel map.
//
// A word is only re-tested when something that its test reads has changed
// since its last test: D0/D1 flag the words whose even / odd columns must be
// tested, set by a new activation in the word and by a change in its 3x3 word
// neighbourhood. An unflagged word would test exactly as before (no simple
// candidate), so skipping it leaves the schedule and its result unchanged.
template <bool LDS>
__device__ __forceinline__ void run_rounds(const Img<LDS>& g, bool thin)
{
    const int rstep = BLOCK / g.WW;  // rows covered per sweep step
    const int my_r = threadIdx.x / g.WW;
    const int my_w = threadIdx.x - my_r * g.WW;
    const bool active = my_r < rstep;
    const uint64_t flip = thin ? 0ull : ~0ull;  // live = M & (S ^ flip)
    const bool has_l = my_w > 0, has_r = my_w + 1 < g.WW;
    // "something changed in round n" lives in chg[n & 1]: written by any
    // changer, read by all after the round's last barrier, and cleared for
    // round n + 1 after the first barrier of round n (when every thread has
    // read the flag of round n - 1)
    __shared__ int chg[2];
    if (threadIdx.x == 0) {
        chg[0] = 0;
        chg[1] = 0;
    }
    __syncthreads();
    for (int round = 0;; ++round) {
        int changed = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int si = s >> 1, sj = s & 1;
            const uint64_t cm = sj ? ODD_COLS : EVEN_COLS;
            auto Dself = sj ? g.D1 : g.D0;
            auto Doth = sj ? g.D0 : g.D1;
            if (active) {
                for (int rr = my_r;; rr += rstep) {
                    const int row = si + 2 * rr;
                    if (row >= g.H)
                        break;
                    const int idx = (si ? g.E : 0) + rr * g.WW + my_w;
                    if (!Dself[idx])
                        continue;
                    Dself[idx] = 0;
                    const uint64_t sc = g.S[idx];
                    const uint64_t live = g.M[idx] & cm & (sc ^ flip);
                    if (!live)
                        continue;
                    // rows row-1 and row+1 live in the other parity half
                    const bool has_u = row > 0, has_d = row + 1 < g.H;
                    const int iu = (si ? 0 : g.E) + (rr - (si ? 0 : 1)) * g.WW + my_w;
                    const int id = (si ? 0 : g.E) + (rr + (si ? 1 : 0)) * g.WW + my_w;
                    const uint64_t u = has_u ? g.S[iu] : 0;
                    const uint64_t ul = has_u && has_l ? g.S[iu - 1] : 0;
                    const uint64_t ur = has_u && has_r ? g.S[iu + 1] : 0;
                    const uint64_t cl = has_l ? g.S[idx - 1] : 0;
                    const uint64_t cr = has_r ? g.S[idx + 1] : 0;
                    const uint64_t d = has_d ? g.S[id] : 0;
                    const uint64_t dl = has_d && has_l ? g.S[id - 1] : 0;
                    const uint64_t dr = has_d && has_r ? g.S[id + 1] : 0;
                    // bit p of E = column p+1, of W = column p-1
                    const uint64_t xE = (sc >> 1) | (cr << 63);
                    const uint64_t xW = (sc << 1) | (cl >> 63);
                    const uint64_t xNE = (u >> 1) | (ur << 63);
                    const uint64_t xNW = (u << 1) | (ul >> 63);
                    const uint64_t xSE = (d >> 1) | (dr << 63);
                    const uint64_t xSW = (d << 1) | (dl >> 63);
                    const uint64_t del = live & simple_bits<uint64_t>(xE, xNE, u, xNW, xW, xSW, d, xSE);
                    if (del) {
                        g.S[idx] = sc ^ del;  // thin clears, thicken sets the bits of del
                        changed = 1;
                        // the other column parity of this word and of the words
                        // beside it; both parities of the three words above and below
                        Doth[idx] = 1;
                        if (has_l)
                            Doth[idx - 1] = 1;
                        if (has_r)
                            Doth[idx + 1] = 1;
                        if (has_u) {
                            g.D0[iu] = 1;
                            g.D1[iu] = 1;
                            if (has_l) {
                                g.D0[iu - 1] = 1;
                                g.D1[iu - 1] = 1;
                            }
                            if (has_r) {
                                g.D0[iu + 1] = 1;
                                g.D1[iu + 1] = 1;
                            }
                        }
                        if (has_d) {
                            g.D0[id] = 1;
                            g.D1[id] = 1;
                            if (has_l) {
                                g.D0[id - 1] = 1;
                                g.D1[id - 1] = 1;
                            }
                            if (has_r) {
                                g.D0[id + 1] = 1;
                                g.D1[id + 1] = 1;
                            }
                        }
                    }
                }
            }
            if (changed)
                chg[round & 1] = 1;
            __syncthreads();
            if (s == 0 && threadIdx.x == 0)
                chg[(round + 1) & 1] = 0;
        }
        if (!chg[round & 1])
            break;
    }
}

}  // namespace hasf_dev
