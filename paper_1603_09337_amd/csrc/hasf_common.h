// Shared host/device definitions of libhasf: the bit-sliced simple-point
// test, level tables for Euclidean balls, and the context structure.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <string>

#include "libhasf.h"

#define HASF_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// Simple-point test (Sec. 2). For (8,4), a point with neighbours x0..x7
// (E NE N NW W SW S SE) is simple iff T = T-bar = 1. Counting, around the
// ring, the background 4-neighbours x_2k whose counter-clockwise successor
// path x_2k+1, x_2k+2 is not all background gives the number of background
// 4-components touching the centre (Yokoi's 8-connectivity number); the
// point is simple exactly when that count is 1 (an isolated point and an
// interior point both give 0). The test is written on words so that it
// evaluates 64 pixels (one per bit) at once; hasf_simple_lut evaluates the
// same function on single bits, and the tests compare that table with an
// independent component-counting table on all 256 codes.
// ---------------------------------------------------------------------------
template <typename T>
HASF_HD T simple_bits(T x0, T x1, T x2, T x3, T x4, T x5, T x6, T x7)
{
    const T t0 = ~x0 & (x1 | x2);
    const T t1 = ~x2 & (x3 | x4);
    const T t2 = ~x4 & (x5 | x6);
    const T t3 = ~x6 & (x7 | x0);
    // exactly one of t0..t3
    return (t0 ^ t1 ^ t2 ^ t3) & ~((t0 & t1) | (t2 & t3));
}

// ---------------------------------------------------------------------------
// Euclidean balls. Offsets (a, b), a, b >= 0, with a^2 + b^2 <= R^2, sorted by
// v = a^2 + b^2: a pixel whose nearest feature lies at row offset +-a and
// column offset +-b has squared distance v. rank(v) = number of sums of two
// squares in [1, v): consecutive distinct values of v are consecutive levels.
// ---------------------------------------------------------------------------
constexpr int HASF_V_MAX = HASF_R_MAX * HASF_R_MAX;

struct BallPairs {
    int n;
    unsigned char a[256];
    unsigned char b[256];
    unsigned short v[256];
    unsigned char rank[256];
};

constexpr bool is_sum_two_squares(int v)
{
    for (int a = 0; a * a <= v; ++a)
        for (int b = 0; a * a + b * b <= v; ++b)
            if (a * a + b * b == v)
                return true;
    return false;
}

constexpr int level_count(int R)  // distinct nonzero squared distances <= R^2
{
    bool hit[HASF_V_MAX + 1] = {};
    for (int a = 0; a <= R; ++a)
        for (int b = 0; a * a + b * b <= R * R; ++b)
            hit[a * a + b * b] = true;
    int c = 0;
    for (int v = 1; v <= R * R; ++v)
        c += hit[v] ? 1 : 0;
    return c;
}

constexpr BallPairs make_ball_pairs(int R)
{
    BallPairs p{};
    bool hit[HASF_V_MAX + 1] = {};
    for (int a = 0; a <= R; ++a)
        for (int b = 0; a * a + b * b <= R * R; ++b)
            hit[a * a + b * b] = true;
    p.n = 0;
    int rk = 0;
    for (int v = 1; v <= R * R; ++v) {
        if (!hit[v])
            continue;
        for (int a = 0; a <= R; ++a)
            for (int b = 0; b <= R; ++b)
                if (a * a + b * b == v) {
                    p.a[p.n] = (unsigned char)a;
                    p.b[p.n] = (unsigned char)b;
                    p.v[p.n] = (unsigned short)v;
                    p.rank[p.n] = (unsigned char)rk;
                    ++p.n;
                }
        ++rk;
    }
    return p;
}

static_assert(level_count(10) == 43, "levels at radius 10");
static_assert(make_ball_pairs(HASF_R_MAX).n <= 256, "ball offsets");
static_assert(level_count(HASF_R_MAX) <= 128, "level counters");
constexpr int HASF_LEVELS_MAX = level_count(HASF_R_MAX);

// Bytes of the state kept per image (LDS when it fits, else global memory):
//   S  the current set as four subfield sub-images: sub-image (si, sj) holds
//      the pixels (2r + si, 2c + sj), 32 columns c per 32-bit word;
//   M  the activated candidates, same layout; its memory also holds R, the
//      row-major view of S (64 columns per 64-bit word) that the distance
//      stages read, while no candidate is active;
//   D  one byte per sub-image word: the word must be re-tested;
//   L  the live words of the running pass.
__host__ __device__ inline size_t state_bytes(int H, int W, bool lds)
{
    const size_t WW = (size_t)(W + 63) / 64, HH = (size_t)(H + 1) / 2;
    const size_t SUB = (HH * WW + 3) & ~(size_t)3;
    // S and M: 4 sub-images of 4-byte words; D: 1 byte per word; the live list
    // of a pass: 2-byte (LDS) or 4-byte (global) word indices
    return 36 * SUB + (lds ? 2 : 4) * SUB;
}

// ---------------------------------------------------------------------------
// Per-image descriptor used by the persistent filter kernel.
// ---------------------------------------------------------------------------
struct ImgDesc {
    uint8_t* X;
    const uint8_t* C;
    long long ld;
    int H, W, r;
    int lds;            // 1: S and M planes in LDS; 0: in gplanes
    uint64_t* gplanes;  // S, M (when lds == 0), A (saved set), K (constraint), D (background constraint)
    uint32_t* ent_idx;  // level entries: word index, levels(r) x words
    uint64_t* ent_msk;  // level entries: candidate bits
    const uint8_t* D;   // background constraint set (same pitch as X) or NULL
    int conn4;          // 1: the (4,8) connectivity pair; 0: (8,4)
    int order;          // 0: HF_i o HC_i at every radius (cutting first); 1: HC_i o HF_i
};

// Control block of one image filtered by a grid of workgroups (device memory,
// zeroed before each launch): the grid barrier (arrival count, generation,
// abort flag), an error word, the pass control words by barrier-epoch parity
// and the level entry counts.
// The context's grid word block (256 bytes): word 0 is the sticky error
// word; from word GRID_COUNTS_OFF on, four uint64 counts summed over grid
// launches: launches, rounds of the level loops, levels activated, grid
// barriers.
constexpr int GRID_COUNTS_OFF = 16;

struct GridCtl {
    unsigned bar_count, pad0[63];
    unsigned bar_gen, pad1[63];
    unsigned abort, err, pad2[62];
    int ctl[2][8];
    unsigned cnt[HASF_LEVELS_MAX];
};

// One grey-level image of a watershed batch (in place); flags: the kernel
// keeps its per-word flags in LDS (else it tests every word of every pass).
struct GreyDesc {
    uint8_t* F;
    long long ld;
    int H, W;
    int flags;
};

// One volume of a 3D batch: the caller's planes and this launch's work planes
// (S, A, K and two distance planes, D * H * W bytes each, then D * H * W
// 32-bit candidate entries).
struct VolDesc {
    uint8_t* X;
    const uint8_t* C;
    int D, H, W, r;
    uint8_t* work;
};

// Control block of one image filtered by row tiles (device memory, zeroed
// before each launch): the grid barrier, an error word, the last round that
// changed one of a tile's own rows (1-based over the launch, kept twice by
// barrier parity), and per phase (4 per radius) and level whether some tile
// has candidates.
struct TileCtl {
    // arrivals (low half) and arrivals that report a change (high half),
    // summed over all barriers
    unsigned long long bar_arrive, pad0[31];
    // barriers completed (low half) and the high half of bar_arrive when the
    // last one completed
    unsigned long long bar_word, pad1[31];
    unsigned abort, err, pad2[62];
    unsigned last_change[2], pad3[62];
    unsigned lev[4 * HASF_R_MAX][HASF_LEVELS_MAX];
};

constexpr int TILE_NT = 1024;  // threads of a tile's workgroup

// Tiling of one image: nr row bands of TH own rows (TH even, >= halo), the
// last one shorter, each cut into nc column tiles of about WW / nc own words
// (64 columns each); a tile keeps up to ER = TH + 2 halo rows and WWb = its
// own words + TILE_HALO_WORDS on each side in LDS. Tile t is row band t / nc,
// column tile t % nc.
struct TilePlan {
    bool ok;
    int TH, ntiles, ER, halo;
    int nr, nc, WWb;
    size_t lds_bytes;     // dynamic LDS of a tile
    size_t planes_bytes;  // Rg, A, K, Dp (row-major), two exchange copies (sub-images)
    size_t ent_words;     // level entry slots per tile: levels(r) x ER x WWb
    size_t idx_bytes, msk_bytes;
    size_t total() const { return planes_bytes + idx_bytes + msk_bytes; }
};

// Halo words (of 64 columns) a column tile keeps on each side: at least the
// passes run between two exchanges (4 x TILE_ROUNDS_MAX_HOST <= 64 columns).
constexpr int TILE_HALO_WORDS = 1;

// Own words [tile_cw0(c), tile_cw0(c + 1)) of column tile c of nc, WW words
// in a row (the same split on the host and on the device)
__host__ __device__ inline int tile_cw0(int c, int nc, int WW)
{
    return (int)(((long long)c * WW) / nc);
}

// Band words of the widest column tile
__host__ __device__ inline int tile_band_words(int nc, int WW)
{
    if (nc <= 1)
        return WW;
    const int own = (WW + nc - 1) / nc;
    const int b = own + 2 * TILE_HALO_WORDS;
    return b < WW ? b : WW;
}

__host__ __device__ inline size_t tile_sub_words(int H, int W)  // one exchange copy: 4 sub-images of 32-bit words
{
    const size_t WW = (size_t)(W + 63) / 64, HH = (size_t)(H + 1) / 2;
    return 4 * ((HH * WW + 3) & ~(size_t)3);
}

// Scratch of one image in the filter kernel: global bytes for the state (when
// it does not fit in LDS), the saved set A and the constraint K, and the level
// entry lists (one slot per word per level).
struct ImageLayout {
    bool lds;
    size_t lds_bytes;     // dynamic LDS the image needs (0 if it is in global memory)
    size_t planes_bytes;  // [state (unless LDS) | A | K | D]
    size_t idx_bytes, msk_bytes;
    size_t total() const { return planes_bytes + idx_bytes + msk_bytes; }
};

__host__ __device__ inline size_t hasf_align256(size_t x) { return (x + 255) / 256 * 256; }

// Raises a kernel's dynamic LDS limit to `bytes` on the current device, once
// per device (bit d of `done` records device d; devices past 63 set it on
// every call). Launchers run on callers' threads and on server threads.
inline hipError_t allow_dyn_lds(const void* fn, int bytes, std::atomic<uint64_t>& done)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    const uint64_t bit = dev >= 0 && dev < 64 ? 1ull << dev : 0ull;
    if (bit && (done.load(std::memory_order_acquire) & bit))
        return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

inline int hasf_levels(int r)
{
    return level_count(r);
}

inline ImageLayout image_layout(int H, int W, int r, size_t lds_cap)
{
    ImageLayout L;
    const size_t WW = (size_t)(W + 63) / 64, NWD = (size_t)H * WW;
    L.lds = hasf_align256(state_bytes(H, W, true)) <= lds_cap;
    const size_t sb = hasf_align256(state_bytes(H, W, L.lds));
    L.lds_bytes = L.lds ? sb : 0;
    L.planes_bytes = hasf_align256((L.lds ? 0 : sb) + 3 * NWD * 8);
    const size_t nlev = (size_t)(r > 0 ? hasf_levels(r) : 1);
    L.idx_bytes = hasf_align256(nlev * NWD * 4);
    L.msk_bytes = hasf_align256(nlev * NWD * 8);
    return L;
}

// Most rounds a tile runs between two exchanges (also in hasf_device.h).
constexpr int TILE_ROUNDS_MAX_HOST = 8;
static_assert(4 * TILE_ROUNDS_MAX_HOST <= 64 * TILE_HALO_WORDS, "a column tile's halo covers the passes between exchanges");


// Tiling of an H x W image at radius r with row bands of TH_req own rows and
// `halo` halo rows (0: the defaults by image size), at most max_tiles tiles in
// all (taller bands when needed),
// each band cut into NC_req column tiles (0: as many as max_tiles allows, at
// least 8 own words each, so that the tiles fill the CUs). Not ok when a band
// of `halo` own rows and its halos does not fit lds_cap bytes of LDS, or when
// the image would be one tile.
inline TilePlan tile_plan(int H, int W, int r, size_t lds_cap, int max_tiles, int TH_req, int halo = 0,
                          int NC_req = 0)
{
    TilePlan P{};
    P.ok = false;
    // the default shape by image size
    const size_t px = (size_t)H * (size_t)W;
    const bool large = px >= HASF_TILE_LARGE_PIXELS, small = px < HASF_TILE_SMALL_PIXELS;
    if (halo == 0)
        halo = large ? HASF_TILE_HALO_LARGE : small ? HASF_TILE_HALO_SMALL : HASF_TILE_HALO_DEFAULT;
    if (TH_req == 0)
        TH_req = large ? HASF_TILE_ROWS_LARGE : small ? HASF_TILE_ROWS_SMALL : HASF_TILE_ROWS_DEFAULT;
    if (halo < 4 || halo > 4 * TILE_ROUNDS_MAX_HOST || (halo & 3) || max_tiles < 2)
        return P;
    P.halo = halo;
    const int WW = (W + 63) / 64;
    const size_t NWD = (size_t)H * WW;
    int th = TH_req;
    th = th < halo ? halo : th;
    th = (th + 1) / 2 * 2;
    int nr = (H + th - 1) / th;
    if (nr > max_tiles) {
        th = (H + max_tiles - 1) / max_tiles;
        th = (th + 1) / 2 * 2;
        nr = (H + th - 1) / th;
    }
    int ncap = max_tiles / nr;
    ncap = ncap < WW ? ncap : WW;
    int nc = NC_req > 0 ? NC_req : WW / 8;
    nc = nc < ncap ? nc : ncap;
    nc = nc < 1 ? 1 : nc;
    const int WWb = tile_band_words(nc, WW);
    const int Wb = nc > 1 ? 64 * WWb : W;  // band width in columns
    int ercap = 0;
    while (ercap < H + 2 * halo && hasf_align256(state_bytes(ercap + 2, Wb, true)) <= lds_cap)
        ercap += 2;
    const int thmax = ((ercap - 2 * halo) / 2) * 2;
    if (thmax < halo)
        return P;
    if (th > thmax) {
        th = thmax;
        nr = (H + th - 1) / th;
        if (nr * nc > max_tiles)
            return P;
    }
    if (nr * nc < 2)
        return P;
    P.ok = true;
    P.TH = th;
    P.nr = nr;
    P.nc = nc;
    P.WWb = WWb;
    P.ntiles = nr * nc;
    P.ER = th + 2 * halo < H ? th + 2 * halo : H;
    P.lds_bytes = hasf_align256(state_bytes(P.ER, Wb, true));
    P.planes_bytes = hasf_align256(4 * NWD * 8) + 2 * hasf_align256(tile_sub_words(H, W) * 4);
    const size_t nlev = (size_t)(r > 0 ? hasf_levels(r) : 1);
    P.ent_words = nlev * (size_t)P.ER * (size_t)WWb;
    P.idx_bytes = hasf_align256((size_t)P.ntiles * P.ent_words * 4);
    P.msk_bytes = hasf_align256((size_t)P.ntiles * P.ent_words * 8);
    return P;
}

// Arguments of the standalone thinning / thickening kernel.
namespace hasf_detail {

struct TopoArgs {
    uint8_t* X;
    const uint8_t* B;  // K (thin) or V (thicken); may be NULL for thin
    long long ld;
    int H, W;
    int thin;
    int conn4;              // 1: the (4,8) pair; 0: (8,4)
    int lds;                // S and M planes in LDS
    const uint32_t* P;      // priorities, pitch W
    uint64_t* planes;       // S, M (when lds == 0), Bp
    uint64_t* bitmap;       // one bit per priority value
    uint32_t* rank_base;    // per bitmap word: number of set bits before it
    uint32_t* hist;         // per level: end offset after the scatter
    uint32_t* ent;          // candidate pixels grouped by level
    unsigned long long nbw; // bitmap words
};

}  // namespace hasf_detail

// host-side context
// How a lone image is filtered: by one workgroup, by row tiles of th own
// rows and `halo` halo rows, or by the grid kernel (state in global memory).
struct LaunchChoice {
    enum Kind { WORKGROUP = 0, TILES = 1, GRID = 2 };
    int kind;
    int th, halo;
    float ms;  // measured time of the choice (0 when not measured)
};

struct hasf_ctx {
    int device;
    hipStream_t stream;
    size_t hbm_budget;
    int num_cu;
    int num_xcd;  // XCDs (accelerator complex dies); workgroups are dealt to them round-robin
    size_t lds_per_block;
    char err[512];
    // growable device scratch
    void* scratch;
    size_t scratch_bytes;
    ImgDesc* d_desc;
    int desc_cap;
    int* d_counter;
    // images of at least this many pixels are filtered by a grid of
    // workgroups: alone (hasf_filter, a batch of one), in batches and served
    size_t grid_min_px, batch_grid_min_px;
    // own rows per tile of the row-tile path for large images (0: default;
    // -1: large images always go to the grid kernel), halo rows per side and
    // column tiles per row band (0: as many as fill the CUs)
    int tile_rows, tile_halo, tile_cols;
    // measured launch choices of lone images by size class, and the file they
    // are kept in (empty: no tuning)
    std::map<uint64_t, LaunchChoice> tune;
    std::string tune_path;
    // sticky device word set by a grid launch whose barrier gave up; read and
    // cleared by hasf_sync when grid work was enqueued since the last check
    unsigned* d_grid_err;
    bool grid_pending;
    // grid images of a batch run on this stream, beside the batch launch
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
    // orders a new stream after the old one in hasf_set_stream
    hipEvent_t ev_switch;
    // pinned staging of a call's descriptors; ev_stage: its last upload
    char* h_stage;
    size_t h_stage_bytes;
    hipEvent_t ev_stage;
};

// Workgroups of the grid that filters one image of nwd 64-bit words: at
// least 8 (one per XCD), about one per 4096 words, at most 16 (more
// workgroups make every grid barrier dearer than the work they take over).
inline int grid_blocks(int nwd, int cap)
{
    int g = (nwd + 4095) / 4096;
    g = g < 8 ? 8 : (g > 16 ? 16 : g);
    return g < cap ? g : (cap > 0 ? cap : 1);
}
