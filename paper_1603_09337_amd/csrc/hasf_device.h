// Device code shared by the libhasf kernels: the bit-packed state of an image,
// packing of byte images, and the subfield rounds of thinning / thickening.
#pragma once

#include <type_traits>

#include "hasf_common.h"

namespace hasf_dev {

constexpr int BLOCK = 512;

// explicit address spaces keep LDS accesses on ds_* and global ones on
// global_* instructions across non-inlined calls
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(1))) uint64_t glb_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) uint32_t glb_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(1))) uint8_t glb_u8;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) int lds_i32;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u4;
typedef __attribute__((address_space(1))) u32x4 glb_u4;
typedef __attribute__((address_space(1))) uint16_t glb_u16;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u32x2 lds_u2;
typedef __attribute__((address_space(1))) u32x2 glb_u2;

enum StageMode {
    HC_THIN = 0,     // features = complement u outside; base = S \ K; saves S into A
    HC_THICKEN = 1,  // features = S; base = A \ S
    HF_THICKEN = 2,  // features = S; base = window \ S; saves S into A
    HF_THIN = 3      // features = complement u outside; base = S \ A
};

// bits 0, 2, 4, ... of x -> bits 0..31
__device__ __forceinline__ uint32_t even_bits(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// bit t of v -> bit 2t
__device__ __forceinline__ uint64_t spread_bits(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

template <bool LDS>
struct Img {
    using P64 = typename std::conditional<LDS, lds_u64*, glb_u64*>::type;
    using P32 = typename std::conditional<LDS, lds_u32*, glb_u32*>::type;
    using P8 = typename std::conditional<LDS, lds_u8*, glb_u8*>::type;
    // list of the live words of a pass (16-bit indices in LDS, 32-bit in global)
    using PL = typename std::conditional<LDS, lds_u16*, glb_u32*>::type;
    P64 R;        // row-major view of the current set (distance stages)
    P32 S;        // current set, four sub-images
    P32 M;        // activated candidates, four sub-images (shares memory with R)
    P8 D;         // per sub-image word: must be re-tested
    PL L;         // live words of the running pass
    lds_i32* ctl; // control words in LDS, see run_rounds
    glb_u64* A;   // set saved before the phase (row-major)
    glb_u64* K;   // constraint set (row-major)
    glb_u64* Dp;  // background constraint set \ X (row-major)
    glb_u32* eidx;
    glb_u64* emsk;
    int H, W, WW, NWD, HH, SUB;
    uint64_t lastmask;  // valid bits of the last word of a row
    bool hasK;
    bool hasD;
    bool conn4;  // the (4,8) pair

    __device__ __forceinline__ int sub(int si, int sj) const { return (si * 2 + sj) * SUB; }
};

// state at `base` (LDS or global), laid out as S | M (= R) | D
template <bool LDS>
__device__ __forceinline__ void bind_state(Img<LDS>& g, void* base)
{
    g.WW = (g.W + 63) >> 6;
    g.NWD = g.H * g.WW;
    g.HH = (g.H + 1) >> 1;
    g.SUB = (g.HH * g.WW + 3) & ~3;
    g.lastmask = (g.W & 63) ? ((1ull << (g.W & 63)) - 1ull) : ~0ull;
    g.S = (typename Img<LDS>::P32)base;
    g.M = g.S + 4 * (size_t)g.SUB;
    g.R = (typename Img<LDS>::P64)g.M;
    g.D = (typename Img<LDS>::P8)(g.M + 4 * (size_t)g.SUB);
    g.L = (typename Img<LDS>::PL)(g.D + 4 * (size_t)g.SUB);
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

// One 64-bit word of the nonzero bytes p[0 .. n) (n <= 64; 16-byte loads
// when vec and n == 64, p then being 16-byte aligned).
__device__ __forceinline__ uint64_t pack_word(const uint8_t* __restrict__ p, int n, bool vec)
{
    uint64_t m = 0;
    if (vec && n == 64) {
        const uint4* xp = reinterpret_cast<const uint4*>(p);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint4 v = xp[j];
            uint64_t bits = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
            m |= bits << (16 * j);
        }
    } else {
        for (int j = 0; j < n; ++j)
            m |= (uint64_t)(p[j] != 0) << j;
    }
    return m;
}

// Bits 0 .. n - 1 of m as bytes 0/1 at p (the same alignment rule).
__device__ __forceinline__ void unpack_word(uint8_t* __restrict__ p, int n, uint64_t m, bool vec)
{
    if (vec && n == 64) {
        uint4* xp = reinterpret_cast<uint4*>(p);
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
        for (int j = 0; j < n; ++j)
            p[j] = (uint8_t)((m >> j) & 1u);
    }
}

// Row-major 64-bit words of the nonzero bytes of X (and of C n X into K when
// K is given): one thread per word. Threads t0, t0 + tn, ... of the caller's
// range (a workgroup, or every workgroup of a grid) share the words.
template <typename PR>
__device__ void pack_rows(const uint8_t* __restrict__ X, const uint8_t* __restrict__ C, long long ld, int H,
                          int W, PR R, glb_u64* K, int t0, int tn)
{
    const int WW = (W + 63) >> 6, NWD = H * WW;
    const bool vec_ok = ((((uintptr_t)X) | (C ? (uintptr_t)C : 0) | (uintptr_t)ld) & 15) == 0;
    for (int q = t0; q < NWD; q += tn) {
        const int row = q / WW;
        const int w = q - row * WW;
        const int c0 = w * 64;
        const int n = min(64, W - c0);
        const uint64_t m = pack_word(X + (long long)row * ld + c0, n, vec_ok);
        R[q] = m;
        if (K)
            K[q] = (C ? pack_word(C + (long long)row * ld + c0, n, vec_ok) : 0ull) & m;
    }
}

// The background constraint set minus the object: D's bits packed into Dp,
// then the bits of X (R, packed by the same threads) cleared.
template <typename PR>
__device__ void pack_background(const uint8_t* __restrict__ D, long long ld, int H, int W, PR R, glb_u64* Dp,
                                int t0, int tn)
{
    pack_rows(D, (const uint8_t*)nullptr, ld, H, W, Dp, (glb_u64*)nullptr, t0, tn);
    const int NWD = H * ((W + 63) >> 6);
    for (int q = t0; q < NWD; q += tn)
        Dp[q] &= ~R[q];
}

template <typename PR>
__device__ void unpack_rows(uint8_t* __restrict__ X, long long ld, int H, int W, PR R, int t0, int tn)
{
    const int WW = (W + 63) >> 6, NWD = H * WW;
    const bool vec_ok = ((((uintptr_t)X) | (uintptr_t)ld) & 15) == 0;
    for (int q = t0; q < NWD; q += tn) {
        const int row = q / WW;
        const int w = q - row * WW;
        const int c0 = w * 64;
        unpack_word(X + (long long)row * ld + c0, min(64, W - c0), R[q], vec_ok);
    }
}

// R -> S (the four sub-images); S -> R
template <bool LDS>
__device__ void rows_to_sub(const Img<LDS>& g, int t0, int tn)
{
    for (int q = t0; q < g.NWD; q += tn) {
        const int row = q / g.WW;
        const int w = q - row * g.WW;
        const uint64_t v = g.R[q];
        const int o = (row >> 1) * g.WW + w;
        g.S[g.sub(row & 1, 0) + o] = even_bits(v);
        g.S[g.sub(row & 1, 1) + o] = even_bits(v >> 1);
    }
}

template <bool LDS>
__device__ void sub_to_rows(const Img<LDS>& g, int t0, int tn)
{
    for (int q = t0; q < g.NWD; q += tn) {
        const int row = q / g.WW;
        const int w = q - row * g.WW;
        const int o = (row >> 1) * g.WW + w;
        g.R[q] = spread_bits(g.S[g.sub(row & 1, 0) + o]) | (spread_bits(g.S[g.sub(row & 1, 1) + o]) << 1);
    }
}

// no candidate active, no word flagged (destroys R)
template <bool LDS>
__device__ void clear_candidates(const Img<LDS>& g, int t0, int tn)
{
    using P32 = typename Img<LDS>::P32;
    const P32 D4 = (P32)g.D;  // 4 * SUB flag bytes, SUB a multiple of 4
    for (int q = t0; q < 4 * g.SUB; q += tn) {
        g.M[q] = 0;
        if (q < g.SUB)
            D4[q] = 0;
    }
}

// Control words (LDS). Every activation and every executed pass gets a
// serial number, uniform across the workgroup and strictly increasing within
// a phase. chg holds the serial of the last pass that changed a pixel;
// prod[s] the serial of the last activation or pass that flagged a word of
// sub-image s; cnt[2] are the shared live-list lengths of alternate passes
// that use one. A pass of sub-image s runs only if prod[s] grew since it last
// ran; a round changed the set iff chg exceeds the serial at the start of
// the round.
//
// prod is kept twice, by the parity of the executed passes. Between the
// barriers that end two executed passes, every wave takes its skip decisions
// (reading one copy) and then runs the next pass, whose changes write the
// other copy. Without the second copy a wave that runs ahead could store
// prod[s] of a later pass while a slower wave has still to decide whether
// to skip pass s (waves of a per-wave pass meet no barrier before their
// stores): it would see the new serial, run a pass the other waves skipped,
// and the workgroup's barriers would go out of step. Each executed pass also
// carries the read copy into the written one (atomic max: values are serials,
// so max is the history), so the next decisions see every earlier store.
// Activations write both copies (no decision is pending while they run).
// chg needs no second copy: it only grows, and a wave can only store it in
// a new round after reading, like every other wave, that the last round
// changed something.
// TILE rounds (see run_rounds) flag a change of the tile's own rows in round
// k at CTL_TCHG + k.
enum { CTL_CHG = 0, CTL_CNT = 2, CTL_PROD = 4, CTL_WORDS = 8, CTL_PROD2 = 8, CTL_TCHG = 12, CTL_LDS_WORDS = 20 };
constexpr int TILE_ROUNDS_MAX = 8;
static_assert(TILE_ROUNDS_MAX == TILE_ROUNDS_MAX_HOST, "rounds between tile exchanges");

// per-phase scheduling state (uniform registers)
struct Sched {
    int serial;       // last serial handed out
    int npass;        // passes with a shared list (selects its length word); grid path: chunks listed
    int consumed[4];  // prod value seen when the sub-image's pass last ran
    int rd;           // workgroup path: offset of the prod copy the next decisions read (0 or 4)
};

// start of a phase; needs a barrier before the first activation
template <bool LDS>
__device__ __forceinline__ void sched_reset(const Img<LDS>& g, Sched& sc)
{
    sc.serial = 0;
    sc.npass = 0;
    for (int k = 0; k < 4; ++k)
        sc.consumed[k] = 0;
    sc.rd = 0;
    if (threadIdx.x < CTL_LDS_WORDS)
        g.ctl[threadIdx.x] = 0;
}

// activate the candidate bits `m` of row-major word (row, w)
template <bool LDS>
__device__ __forceinline__ void activate_row_word(const Img<LDS>& g, int row, int w, uint64_t m, int serial)
{
    const int o = (row >> 1) * g.WW + w;
    const uint32_t e = even_bits(m), od = even_bits(m >> 1);
    if (e) {
        const int q = g.sub(row & 1, 0) + o;
        __hip_atomic_fetch_or(g.M + q, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        g.D[q] = 1;
        g.ctl[CTL_PROD + (row & 1) * 2] = serial;
        g.ctl[CTL_PROD2 + (row & 1) * 2] = serial;
    }
    if (od) {
        const int q = g.sub(row & 1, 1) + o;
        __hip_atomic_fetch_or(g.M + q, od, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        g.D[q] = 1;
        g.ctl[CTL_PROD + (row & 1) * 2 + 1] = serial;
        g.ctl[CTL_PROD2 + (row & 1) * 2 + 1] = serial;
    }
}

// activate pixel (i, j)
template <bool LDS>
__device__ __forceinline__ void activate_pixel(const Img<LDS>& g, int i, int j, int serial)
{
    const int c = j >> 1;
    const int q = g.sub(i & 1, j & 1) + (i >> 1) * g.WW + (c >> 5);
    __hip_atomic_fetch_or(g.M + q, 1u << (c & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    g.D[q] = 1;
    g.ctl[CTL_PROD + (i & 1) * 2 + (j & 1)] = serial;
    g.ctl[CTL_PROD2 + (i & 1) * 2 + (j & 1)] = serial;
}

// Orders the stores a wave made before it against the loads its lanes make
// after it (a wave-private list written by some lanes and read by others).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive prefix over the wave of v in [0, 7]; *total = sum over the wave.
// Bit-sliced with ballots: no cross-lane data movement through LDS.
__device__ __forceinline__ unsigned wave_prefix(unsigned v, unsigned* total)
{
    const uint64_t lt = lanemask_lt();
    const uint64_t b0 = __ballot(v & 1u), b1 = __ballot(v & 2u), b2 = __ballot(v & 4u);
    *total = (unsigned)(__popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2));
    return (unsigned)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt));
}

// Pointers of one subfield pass: the pass's own sub-image (si, sj) and the
// three it reads (E/W: same rows, other column parity; N/S: other row parity,
// same columns; diagonals: the fourth), with their re-test flags.
template <bool LDS>
struct PassPtrs {
    typename Img<LDS>::P32 Ss, Ms, Sx, Sy, Sxy;
    typename Img<LDS>::P8 Dx, Dy, Dxy;
};

template <bool LDS>
__device__ __forceinline__ PassPtrs<LDS> pass_ptrs(const Img<LDS>& g, int si, int sj)
{
    const int so = 1 - si, co = 1 - sj;
    PassPtrs<LDS> p;
    p.Ss = g.S + g.sub(si, sj);
    p.Ms = g.M + g.sub(si, sj);
    p.Sx = g.S + g.sub(si, co);
    p.Sy = g.S + g.sub(so, sj);
    p.Sxy = g.S + g.sub(so, co);
    p.Dx = g.D + g.sub(si, co);
    p.Dy = g.D + g.sub(so, sj);
    p.Dxy = g.D + g.sub(so, co);
    return p;
}

// The words a subfield-pass test of word idx reads (row rr of sub-image
// (si, sj), WW words per row, H image rows): its own S and M words and the
// neighbouring words of the other three sub-images.
struct WordNbhd {
    int idx, iN, iS;
    bool hasL, hasR, hasN, hasS;
    uint32_t scw, m, xc, xl, xr, nn, sv, nc, nl, nr, dc, dl, dr;
};

template <bool LDS>
__device__ __forceinline__ WordNbhd load_word(const PassPtrs<LDS>& p, int idx, int rr, int si, int WW, int H)
{
    WordNbhd n;
    const int my_w = idx - rr * WW;
    n.idx = idx;
    n.hasL = my_w > 0;
    n.hasR = my_w + 1 < WW;
    const int row = 2 * rr + si;
    n.hasN = row > 0;
    n.hasS = row + 1 < H;
    n.iN = (si ? rr : rr - 1) * WW + my_w;  // row - 1 in the other parity
    n.iS = (si ? rr + 1 : rr) * WW + my_w;  // row + 1
    // Every load is issued, at an index inside the sub-image (a missing
    // neighbour row or column reads the word's own index, or its row), and a
    // missing neighbour's value is then replaced by 0: no branch per load.
    // iN and iS themselves become such indices (apply_word flags through
    // them: a flag on a word whose inputs did not change only re-tests it).
    const int l = n.hasL ? 1 : 0, r = n.hasR ? 1 : 0;
    n.iN = n.hasN ? n.iN : (n.hasS ? n.iS : idx);
    n.iS = n.hasS ? n.iS : n.iN;
    const uint32_t xl = p.Sx[idx - l], xr = p.Sx[idx + r];
    const uint32_t nn = p.Sy[n.iN], sv = p.Sy[n.iS];
    const uint32_t nc = p.Sxy[n.iN], nl = p.Sxy[n.iN - l], nr = p.Sxy[n.iN + r];
    const uint32_t dc = p.Sxy[n.iS], dl = p.Sxy[n.iS - l], dr = p.Sxy[n.iS + r];
    n.scw = p.Ss[idx];
    n.m = p.Ms[idx];
    n.xc = p.Sx[idx];
    n.xl = n.hasL ? xl : 0u;
    n.xr = n.hasR ? xr : 0u;
    n.nn = n.hasN ? nn : 0u;
    n.sv = n.hasS ? sv : 0u;
    n.nc = n.hasN ? nc : 0u;
    n.nl = n.hasN && n.hasL ? nl : 0u;
    n.nr = n.hasN && n.hasR ? nr : 0u;
    n.dc = n.hasS ? dc : 0u;
    n.dl = n.hasS && n.hasL ? dl : 0u;
    n.dr = n.hasS && n.hasR ? dr : 0u;
    return n;
}

// Flips the simple live candidates of a loaded word (thinning deletes,
// thickening adds: live = M & (S ^ flip)) and flags every word whose test
// reads a changed word. Returns whether a pixel changed. conn4: the (4,8)
// pair, whose simple points are the (8,4) ones of the complemented
// neighbourhood (the outside of the window, background, becomes object).
template <bool LDS>
__device__ __forceinline__ bool apply_word(const PassPtrs<LDS>& p, const WordNbhd& n, int sj, uint32_t flip,
                                           bool conn4 = false)
{
    const uint32_t live = n.m & (n.scw ^ flip);
    // column c of this sub-image is image column 2c + sj; its east neighbour
    // is column c (sj = 0) or c + 1 (sj = 1) of the other column parity, its
    // west one c - 1 or c
    uint32_t e, w, ne, nw2, se, sw;
    if (sj == 0) {
        e = n.xc;
        w = (n.xc << 1) | (n.xl >> 31);
        ne = n.nc;
        nw2 = (n.nc << 1) | (n.nl >> 31);
        se = n.dc;
        sw = (n.dc << 1) | (n.dl >> 31);
    } else {
        e = (n.xc >> 1) | (n.xr << 31);
        w = n.xc;
        ne = (n.nc >> 1) | (n.nr << 31);
        nw2 = n.nc;
        se = (n.dc >> 1) | (n.dr << 31);
        sw = n.dc;
    }
    uint32_t nn = n.nn, sv = n.sv;
    if (conn4) {
        e = ~e;
        ne = ~ne;
        nn = ~nn;
        nw2 = ~nw2;
        w = ~w;
        sw = ~sw;
        sv = ~sv;
        se = ~se;
    }
    const uint32_t del = live & simple_bits<uint32_t>(e, ne, nn, nw2, w, sw, sv, se);
    if (!del)
        return false;
    // the words that read this one, flagged without branches: a missing
    // neighbour column or row maps to a word flagged anyway (load_word), or,
    // for a one-row image, to a word of an empty sub-image
    const int idx = n.idx, iN = n.iN, iS = n.iS;
    const int l = n.hasL ? 1 : 0, r = n.hasR ? 1 : 0;
    p.Ss[idx] = n.scw ^ del;
    p.Dx[idx] = 1;
    p.Dx[idx - l] = 1;
    p.Dx[idx + r] = 1;
    p.Dy[iN] = 1;
    p.Dxy[iN] = 1;
    p.Dxy[iN - l] = 1;
    p.Dxy[iN + r] = 1;
    p.Dy[iS] = 1;
    p.Dxy[iS] = 1;
    p.Dxy[iS - l] = 1;
    p.Dxy[iS + r] = 1;
    return true;
}

// Tests the activated candidates of word idx (row rr of sub-image (si, sj))
// and flips the simple ones; see load_word and apply_word.
template <bool LDS>
__device__ __forceinline__ bool test_word(const PassPtrs<LDS>& p, int idx, int rr, int si, int sj, int WW, int H,
                                          uint32_t flip, bool conn4 = false)
{
    return apply_word(p, load_word(p, idx, rr, si, WW, H), sj, flip, conn4);
}

// Rounds of the four subfield passes (even,even) (even,odd) (odd,even)
// (odd,odd) until a round changes nothing. A pass tests, on the state left by
// the previous pass, the activated candidates of its subfield and flips the
// simple ones (thinning deletes, thickening adds). Two points of one subfield
// are never 8-adjacent, so a pass is a pure data-parallel map: it writes only
// its own sub-image and reads the other three, whose pixels are its points'
// neighbours (E/W: same rows, other column parity; N/S: other row parity,
// same columns; diagonals: the fourth sub-image).
//
// A word is only re-tested when something its test reads has changed since
// its last test: D flags a word on a new activation in it and on a change in
// a word it reads. An unflagged word would test exactly as before (no simple
// candidate), so skipping it leaves the schedule and its result unchanged.
// A pass only clears the flags of its own sub-image and only sets flags of
// the other three, so flags need no atomics. A pass first collects its
// flagged live words into a list (4 flags per thread per load), then tests
// the list densely; a pass whose sub-image has no flagged word is skipped.
// A sub-image of at most 2 NT words is instead split into one 128-word chunk
// per wave, and each wave lists and tests its own chunk's words, which saves
// the workgroup barrier between listing and testing. In a tile (TILE) a
// sub-image of at most NT words is tested one word per thread in place, with
// no list at all.
// NT: the workgroup size (threads) the caller is launched with.
//
// TILE: the state is one tile of a larger image (its own pixels plus halo
// rows and words whose values a neighbouring tile owns). Exactly `nrounds`
// (at most TILE_ROUNDS_MAX) rounds run, since the caller decides when the
// level ends over all tiles, and the result is the number k of rounds run
// until the last one that changed one of the tile's own pixels (rows
// [ilo, ihi), words [wlo, whi)) (0: none did).
// Otherwise the result is 0.
template <bool LDS, int NT = BLOCK, bool TILE = false>
__device__ __forceinline__ int run_rounds(const Img<LDS>& g, bool thin, Sched& sc, int nrounds = 0, int ilo = 0,
                                          int ihi = 0, int wlo = 0, int whi = 0)
{
    const int WW = g.WW;
    const float invWW = 1.0f / (float)WW;
    // row of a word index: in LDS (index < 2^16, WW <= 1024) a multiply by
    // ceil(2^32 / WW) taking the high half is exact (WW = 1, whose factor does
    // not fit 32 bits, is the index itself); in global memory the float
    // estimate is corrected by one step either way
    const uint32_t magic = 0xFFFFFFFFu / (uint32_t)WW + 1u;
    auto row_of = [&](int idx) {
        if constexpr (LDS) {
            return WW == 1 ? idx : (int)__umulhi((uint32_t)idx, magic);
        } else {
            int rr = (int)((float)idx * invWW);
            if (rr * WW > idx)
                --rr;
            else if ((rr + 1) * WW <= idx)
                ++rr;
            return rr;
        }
    };
    const uint32_t flip = thin ? 0u : ~0u;  // live = M & (S ^ flip)
    lds_i32* chg = g.ctl + CTL_CHG;
    lds_i32* lcnt = g.ctl + CTL_CNT;
    if constexpr (TILE) {
        if (threadIdx.x < TILE_ROUNDS_MAX)
            g.ctl[CTL_TCHG + threadIdx.x] = 0;
        __syncthreads();
    }
    for (int rnd = 0;; ++rnd) {
        if (TILE && rnd == nrounds)
            break;
        const int round_start = sc.serial;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            // decisions read one copy of prod, the pass writes the other
            const lds_i32* prod_rd = g.ctl + CTL_PROD + sc.rd;
            lds_i32* prod = g.ctl + CTL_PROD + (sc.rd ^ 4);
            const int p = prod_rd[s];
            // in place (TILE, a sub-image of at most NT words): this thread's
            // flag is loaded with the skip word (and with the four words the
            // pass carries forward into prod), in one LDS round trip; the
            // empty asm keeps the compiler from sinking the loads behind the
            // skip decision. The flag is the one the last executed pass left
            // behind its barrier.
            unsigned f1 = 0;
            int pr = 0;
            if constexpr (LDS && TILE) {
                const int nw1 = ((g.H - (s >> 1) + 1) >> 1) * WW;
                if (nw1 <= NT && (int)threadIdx.x < nw1)
                    f1 = g.D[g.sub(s >> 1, s & 1) + (int)threadIdx.x];
                if (threadIdx.x < 4)
                    pr = prod_rd[threadIdx.x];
                asm volatile("" ::"v"(f1), "v"(p), "v"(pr));
            }
            if (p <= sc.consumed[s])
                continue;  // nothing flagged in this sub-image: the pass would change nothing
            sc.consumed[s] = p;
            const int ser = ++sc.serial;
            if (threadIdx.x < 4)
                __hip_atomic_fetch_max(prod + threadIdx.x, (LDS && TILE) ? pr : prod_rd[threadIdx.x],
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int si = s >> 1, sj = s & 1;
            const int so = 1 - si, co = 1 - sj;
            const auto Ss = g.S + g.sub(si, sj);
            const auto Ms = g.M + g.sub(si, sj);
            const auto Ds = g.D + g.sub(si, sj);
            const int rows = (g.H - si + 1) >> 1;
            const int nw = rows * WW;
            const PassPtrs<LDS> pp = pass_ptrs(g, si, sj);
            bool changed_here = false;
            bool changed_own = false;  // TILE: a change in rows [ilo, ihi), words [wlo, whi)
            auto test = [&](int idx) {
                const int rr = row_of(idx);
                const bool c = test_word(pp, idx, rr, si, sj, WW, g.H, flip, g.conn4);
                changed_here |= c;
                if constexpr (TILE) {
                    const int w = idx - rr * WW;
                    changed_own |= c && 2 * rr + si >= ilo && 2 * rr + si < ihi && w >= wlo && w < whi;
                }
            };
            if (LDS && TILE && nw <= NT) {
                // one word per thread (its flag loaded above), tested in
                // place when flagged: no listing, so a pass is one round trip
                // for the skip word and the flags and one for the test (a
                // test writes only its own word of S and flags of the other
                // three sub-images)
                const int b = (int)threadIdx.x;
                if (b < nw && f1) {
                    Ds[b] = 0;
                    test(b);  // loads M and S with the neighbours: no live candidate, no change
                }
            } else if (nw <= 2 * NT) {
                // one chunk of 128 words per wave, listed at L[w0 ..] and
                // tested by the same wave: a test writes only its own word of
                // S and flags of the other three sub-images, and a wave's
                // listing reads only its own chunk's flags, M and S, so no
                // workgroup barrier is needed between them. The two words'
                // M and S are loaded with their flags (b0 is even and below
                // nw <= SUB, a multiple of 4, so both words lie in the
                // sub-image); the list holds at most the chunk's words below
                // nw.
                using U2 = typename std::conditional<LDS, const lds_u2*, const glb_u2*>::type;
                using F2 = typename std::conditional<LDS, lds_u16*, glb_u16*>::type;
                const int lane = (int)(threadIdx.x & 63);
                const int w0 = 2 * (int)(threadIdx.x & ~63u);
                const int b0 = w0 + 2 * lane;
                unsigned f2 = 0;
                u32x2 m2 = {0u, 0u}, s2 = m2;
                if (b0 < nw) {
                    f2 = *(F2)(Ds + b0);
                    m2 = *(U2)(Ms + b0);
                    s2 = *(U2)(Ss + b0);
                }
                // a wave none of whose 128 words is flagged lists nothing
                if (__ballot(f2 != 0u) != 0) {
                    unsigned nl = 0;
                    int q0 = 0, q1 = 0;
                    if (f2) {
                        *(F2)(Ds + b0) = (uint16_t)0;
                        if ((f2 & 0xFFu) && (m2.x & (s2.x ^ flip))) {
                            q0 = b0;
                            nl = 1;
                        }
                        if ((f2 >> 8) && b0 + 1 < nw && (m2.y & (s2.y ^ flip))) {
                            if (nl) q1 = b0 + 1;
                            else q0 = b0 + 1;
                            ++nl;
                        }
                    }
                    unsigned tot;
                    const unsigned off = wave_prefix(nl, &tot);
                    if (tot) {
                        const auto Lw = g.L + w0;
                        if (nl > 0) Lw[off] = q0;
                        if (nl > 1) Lw[off + 1] = q1;
                        wave_sync();
                        for (int t = lane; t < (int)tot; t += 64)
                            test((int)Lw[t]);
                    }
                }
            } else {
                lds_i32* cnt = lcnt + (sc.npass & 1);
                // collect: flagged words whose activated candidates are still live;
                // every lane runs the same number of iterations (wave-wide prefix).
                // The four words' M and S are loaded with their flags, flagged or
                // not, so the live test waits for one round trip, not three (b0 is
                // a multiple of 4 below nw <= SUB, and SUB is a multiple of 4, so
                // the four words lie in the sub-image)
                using U4 = typename std::conditional<LDS, const lds_u4*, const glb_u4*>::type;
                const int niter = (nw + 4 * NT - 1) / (4 * NT);
                for (int it = 0; it < niter; ++it) {
                    const int b0 = 4 * threadIdx.x + it * 4 * NT;
                    unsigned f4 = 0;
                    u32x4 m4 = {0u, 0u, 0u, 0u}, s4 = m4;
                    if (b0 < nw) {
                        f4 = *(const typename std::conditional<LDS, lds_u32*, glb_u32*>::type)(Ds + b0);
                        m4 = *(U4)(Ms + b0);
                        s4 = *(U4)(Ss + b0);
                    }
                    // a wave none of whose 256 words is flagged lists nothing
                    if (__ballot(f4 != 0u) == 0)
                        continue;
                    // bit j of keep: word b0 + j is flagged, inside the
                    // sub-image and has live candidates
                    const int rem = nw - b0;
                    const uint32_t inside = rem >= 4 ? 0xFu : (rem > 0 ? (1u << rem) - 1u : 0u);
                    const uint32_t lv = (uint32_t)((m4.x & (s4.x ^ flip)) != 0u) |
                                        ((uint32_t)((m4.y & (s4.y ^ flip)) != 0u) << 1) |
                                        ((uint32_t)((m4.z & (s4.z ^ flip)) != 0u) << 2) |
                                        ((uint32_t)((m4.w & (s4.w ^ flip)) != 0u) << 3);
                    const uint32_t keep = nz4(f4) & inside & lv;
                    if (f4)
                        *(typename std::conditional<LDS, lds_u32*, glb_u32*>::type)(Ds + b0) = 0u;
                    const unsigned nl = (unsigned)__popc(keep);
                    unsigned tot;
                    const unsigned off = wave_prefix(nl, &tot);
                    unsigned base = 0;
                    if (tot) {
                        if ((threadIdx.x & 63) == 0)
                            base = (unsigned)__hip_atomic_fetch_add(cnt, (int)tot, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
                        base = (unsigned)__builtin_amdgcn_readfirstlane((int)base) + off;
                        if (nl) {
                            // the k-th listed word is the k-th set bit of keep;
                            // entries past nl rewrite the last one with the
                            // same value, so the four stores need no branch
                            const uint32_t k1 = keep & (keep - 1u), k2 = k1 & (k1 - 1u), k3 = k2 & (k2 - 1u);
                            const int j0 = __ffs(keep) - 1;
                            const int j1 = k1 ? __ffs(k1) - 1 : j0;
                            const int j2 = k2 ? __ffs(k2) - 1 : j1;
                            const int j3 = k3 ? __ffs(k3) - 1 : j2;
                            const unsigned last = nl - 1u;
                            g.L[base] = b0 + j0;
                            g.L[base + min(1u, last)] = b0 + j1;
                            g.L[base + min(2u, last)] = b0 + j2;
                            g.L[base + min(3u, last)] = b0 + j3;
                        }
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0)
                    lcnt[(sc.npass + 1) & 1] = 0;  // every thread read it one pass ago
                const int n = *cnt;
                // test the listed words
                for (int t = threadIdx.x; t < n; t += NT)
                    test((int)g.L[t]);
                ++sc.npass;
            }
            // one lane per wave records the change (a same-address store from
            // many lanes would be serialised)
            {
                const uint64_t chm = __ballot(changed_here);
                if (chm && (int)(threadIdx.x & 63) == __ffsll((long long)chm) - 1) {
                    if (!TILE)
                        *chg = ser;
                    prod[si * 2 + co] = ser;
                    if (g.H > 1) {
                        prod[so * 2 + sj] = ser;
                        prod[so * 2 + co] = ser;
                    }
                }
                if constexpr (TILE) {
                    const uint64_t com = __ballot(changed_own);
                    if (com && (int)(threadIdx.x & 63) == __ffsll((long long)com) - 1)
                        g.ctl[CTL_TCHG + rnd] = 1;
                }
            }
            __syncthreads();
            sc.rd ^= 4;
        }
        // a round changed nothing (and the level is done) iff no pass of it
        // stored its serial in chg; a round without any pass changes nothing
        if (!TILE && *chg <= round_start)
            break;
        // TILE: a round that ran no pass leaves prod as it found it, so every
        // later round of the epoch would skip all its passes too
        if (TILE && sc.serial == round_start)
            break;
    }
    // The skip decisions after the last executed pass read prod and chg with
    // no barrier behind them. The caller's next activation writes prod: a
    // wave that got there first would make a slower wave see a new serial,
    // run a pass the others skipped and leave the workgroup's barriers out
    // of step. Every wave finishes its decisions before anyone goes on.
    __syncthreads();
    int last = 0;
    if constexpr (TILE) {
        for (int k = 0; k < nrounds; ++k)
            if (g.ctl[CTL_TCHG + k])
                last = k + 1;
    }
    return last;
}

}  // namespace hasf_dev
