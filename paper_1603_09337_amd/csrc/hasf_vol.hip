// HASF on 3D binary volumes with 26-connected objects and a 6-connected
// background. The paper smooths 2D and 3D objects (Sec. 1) and applies its
// distance transforms to 3D images (Sec. 4.1); the operators are those of
// Sec. 2 with 3D Euclidean balls and the 3D topological numbers:
//   a voxel x is simple iff T26 = 1 and Tbar6 = 1, where T26 is the number
//   of 26-components of the object voxels of its 26-neighbourhood and Tbar6
//   the number of 6-components of the background voxels of its
//   18-neighbourhood that contain one of its six face neighbours.
// Thinning and thickening follow the 2D schedule with eight subfields: levels
// of increasing squared distance, and inside a level rounds of eight passes
// over the parity classes (z mod 2, y mod 2, x mod 2) in lexicographic order
// until a round changes nothing; two voxels of one class are never
// 26-adjacent, so a pass is a data-parallel map.
//
// One workgroup filters one volume at a time (a persistent queue over the
// batch). The state is byte planes in global memory: S (the set), A (the set
// saved before a cutting or a filling), K (the constraint set), and two
// distance planes. Distances are only ever compared with i^2 or used to order
// candidates within i^2, so the squared distance is computed saturated at
// i^2 + 1, separably over windows of +-i voxels along x, then y, then z
// (exact for every value up to i^2); i <= 15 keeps it in one byte.
#include <atomic>

#include "hasf_common.h"

namespace {

constexpr int VOL_NT = 1024;
constexpr uint8_t VFAR = 255;  // "more than i^2" (i^2 + 1 <= 226 < 255)

// neighbour b = 0..25: offset (dz, dy, dx) of {-1,0,1}^3 without the centre,
// lexicographic in (dz, dy, dx); the adjacency masks among the neighbours
struct VolTables {
    uint32_t adj26[26], adj6[26];
    uint32_t n18, face;
};

constexpr VolTables make_vol_tables()
{
    VolTables t{};
    int off[26][3] = {};
    int b = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dz && !dy && !dx)
                    continue;
                off[b][0] = dz;
                off[b][1] = dy;
                off[b][2] = dx;
                ++b;
            }
    for (int a = 0; a < 26; ++a) {
        const int l1a = (off[a][0] < 0 ? -off[a][0] : off[a][0]) + (off[a][1] < 0 ? -off[a][1] : off[a][1]) +
                        (off[a][2] < 0 ? -off[a][2] : off[a][2]);
        if (l1a <= 2)
            t.n18 |= 1u << a;
        if (l1a == 1)
            t.face |= 1u << a;
        for (int c = 0; c < 26; ++c) {
            if (a == c)
                continue;
            int linf = 0, l1 = 0;
            for (int k = 0; k < 3; ++k) {
                const int d = off[a][k] - off[c][k] < 0 ? off[c][k] - off[a][k] : off[a][k] - off[c][k];
                linf = d > linf ? d : linf;
                l1 += d;
            }
            if (linf == 1)
                t.adj26[a] |= 1u << c;
            if (l1 == 1)
                t.adj6[a] |= 1u << c;
        }
    }
    return t;
}

__constant__ VolTables VT = make_vol_tables();

// the component of `set` that contains the voxels of `seed`
__device__ __forceinline__ uint32_t grow(uint32_t seed, uint32_t set, const uint32_t* adj)
{
    uint32_t c = seed;
    for (;;) {
        uint32_t g = c, m = c;
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            g |= adj[b];
        }
        g &= set;
        if (g == c)
            return c;
        c = g;
    }
}

// T26 = 1 and Tbar6 = 1 for the neighbourhood code
__device__ __forceinline__ bool simple26(uint32_t code)
{
    if (code == 0)
        return false;  // T26 = 0
    const uint32_t c = grow(code & (0u - code), code, VT.adj26);
    if (c != code)
        return false;  // more than one object component
    const uint32_t bg = ~code & VT.n18;
    const uint32_t facebg = bg & VT.face;
    if (!facebg)
        return false;  // Tbar6 = 0
    const uint32_t c6 = grow(facebg & (0u - facebg), bg, VT.adj6);
    return (facebg & ~c6) == 0;  // every background face neighbour in that one component
}

struct Vol {
    uint8_t* S;
    uint8_t* A;
    uint8_t* K;
    uint8_t* G;  // distance work plane
    uint8_t* P;  // squared distance, saturated (VFAR beyond i^2)
    uint32_t* E; // the phase's candidates by (parity class, level)
    int D, H, W;
    long long N;
};

__device__ __forceinline__ uint32_t vol_code(const Vol& v, int z, int y, int x)
{
    uint32_t code = 0;
    int b = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dz && !dy && !dx)
                    continue;
                const int zz = z + dz, yy = y + dy, xx = x + dx;
                if (zz >= 0 && zz < v.D && yy >= 0 && yy < v.H && xx >= 0 && xx < v.W &&
                    v.S[((long long)zz * v.H + yy) * v.W + xx])
                    code |= 1u << b;
                ++b;
            }
    return code;
}

// Squared distance, saturated, to the feature voxels (frame: not in S, and
// every voxel outside the box; else: in S), into v.P. Three separable passes
// over windows of +-i.
__device__ void vol_distance(const Vol& v, int i, bool frame)
{
    const int r2 = i * i;
    // along x: feature test on S directly
    for (long long q = threadIdx.x; q < v.N; q += VOL_NT) {
        const int x = (int)(q % v.W);
        const long long row = q - x;
        int best = VFAR;
        for (int d = -i; d <= i; ++d) {
            const int xx = x + d;
            bool f;
            if (xx < 0 || xx >= v.W)
                f = frame;
            else
                f = frame ? !v.S[row + xx] : v.S[row + xx] != 0;
            if (f && d * d < best)
                best = d * d;
        }
        v.G[q] = (uint8_t)(best > r2 ? VFAR : best);
    }
    __syncthreads();
    // along y, then z: (offset)^2 + previous; outside the box: 0 with the frame
    for (int pass = 0; pass < 2; ++pass) {
        const uint8_t* src = pass == 0 ? v.G : v.P;
        uint8_t* dst = pass == 0 ? v.P : v.G;
        for (long long q = threadIdx.x; q < v.N; q += VOL_NT) {
            const int x = (int)(q % v.W);
            const long long zy = q / v.W;
            const int y = (int)(zy % v.H), z = (int)(zy / v.H);
            const int t = pass == 0 ? y : z, len = pass == 0 ? v.H : v.D;
            const long long stride = pass == 0 ? (long long)v.W : (long long)v.W * v.H;
            int best = VFAR;
            for (int d = -i; d <= i; ++d) {
                const int tt = t + d;
                int g;
                if (tt < 0 || tt >= len)
                    g = frame ? 0 : VFAR;
                else
                    g = src[q + d * stride];
                if (g != VFAR && d * d + g < best)
                    best = d * d + g;
            }
            dst[q] = (uint8_t)(best > r2 ? VFAR : best);
        }
        __syncthreads();
    }
    // the result of the z pass is in G: move it to P
    for (long long q = threadIdx.x; q < v.N; q += VOL_NT)
        v.P[q] = v.G[q];
    __syncthreads();
}

// candidates of the phase: 0 cutting/thin, 1 cutting/thicken, 2 filling/thicken, 3 filling/thin
__device__ __forceinline__ bool vol_cand(const Vol& v, long long q, int mode)
{
    const bool s = v.S[q] != 0;
    switch (mode) {
    case 0: return s && !v.K[q];
    case 1: return !s && v.A[q];
    case 2: return !s;
    default: return s && !v.A[q];
    }
}

// parity class of a voxel: (z mod 2, y mod 2, x mod 2) in lexicographic order
__device__ __forceinline__ int vol_class(const Vol& v, long long q)
{
    const int x = (int)(q % v.W);
    const long long zy = q / v.W;
    const int y = (int)(zy % v.H), z = (int)(zy / v.H);
    return ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
}

// One phase at radius i. The candidates within i^2 are listed once, sorted
// by (parity class, level) with a counting sort, so that the candidates of
// class c at levels <= d are one contiguous run of the list; a pass of level
// d over class c then visits that run only (the voxels that are not, or no
// longer, candidates fail the test at once).
__device__ void vol_phase(const Vol& v, int i, int mode, unsigned* cnt, unsigned* off, int* s_flag)
{
    const bool thin = mode == 0 || mode == 3;
    if (mode == 0 || mode == 2) {
        for (long long q = threadIdx.x; q < v.N; q += VOL_NT)
            v.A[q] = v.S[q];
    }
    vol_distance(v, i, thin);
    const int r2 = i * i;
    const int nl = r2 + 1;  // levels 0..i^2
    const int nk = 8 * nl;  // keys: class * nl + level
    for (int k = threadIdx.x; k < nk; k += VOL_NT)
        cnt[k] = 0;
    __syncthreads();
    for (long long q = threadIdx.x; q < v.N; q += VOL_NT)
        if (v.P[q] != VFAR && vol_cand(v, q, mode))
            atomicAdd(cnt + vol_class(v, q) * nl + v.P[q], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned o = 0;
        for (int k = 0; k < nk; ++k) {
            off[k] = o;
            o += cnt[k];
            cnt[k] = 0;  // becomes the fill count of the key
        }
        off[nk] = o;
    }
    __syncthreads();
    for (long long q = threadIdx.x; q < v.N; q += VOL_NT)
        if (v.P[q] != VFAR && vol_cand(v, q, mode)) {
            const int k = vol_class(v, q) * nl + v.P[q];
            v.E[off[k] + atomicAdd(cnt + k, 1u)] = (uint32_t)q;
        }
    __syncthreads();
    for (int d = 0; d <= r2; ++d) {
        bool any_level = false;
        for (int c = 0; c < 8; ++c)
            any_level |= off[c * nl + d + 1] > off[c * nl + d];
        if (!any_level)
            continue;  // uniform: no candidate at this level
        for (;;) {
            if (threadIdx.x == 0)
                *s_flag = 0;
            __syncthreads();
            for (int c = 0; c < 8; ++c) {
                const unsigned t0 = off[c * nl], t1 = off[c * nl + d + 1];
                bool changed = false;
                for (unsigned t = t0 + threadIdx.x; t < t1; t += VOL_NT) {
                    const long long q = v.E[t];
                    if (!vol_cand(v, q, mode))
                        continue;  // changed in an earlier pass of this phase
                    const int x = (int)(q % v.W);
                    const long long zy = q / v.W;
                    const int y = (int)(zy % v.H), z = (int)(zy / v.H);
                    if (simple26(vol_code(v, z, y, x))) {
                        v.S[q] = thin ? 0 : 1;
                        changed = true;
                    }
                }
                if (changed)
                    *s_flag = 1;
                // the pass's writes before the next pass reads them
                __threadfence_block();
                __syncthreads();
            }
            const int any = *s_flag;
            __syncthreads();
            if (!any)
                break;
        }
    }
}

}  // namespace

// Each workgroup claims volumes in queue order until none is left.
__global__ __launch_bounds__(VOL_NT) void hasf_vol_kernel(const VolDesc* __restrict__ desc, int n,
                                                          int* __restrict__ next)
{
    __shared__ unsigned cnt[8 * (HASF_R_MAX * HASF_R_MAX + 1)];
    __shared__ unsigned off[8 * (HASF_R_MAX * HASF_R_MAX + 1) + 1];
    __shared__ int s_img, s_flag;
    for (;;) {
        if (threadIdx.x == 0)
            s_img = atomicAdd(next, 1);
        __syncthreads();
        const int img = s_img;
        __syncthreads();
        if (img >= n)
            break;
        const VolDesc& d = desc[img];
        Vol v;
        v.D = d.D;
        v.H = d.H;
        v.W = d.W;
        v.N = (long long)d.D * d.H * d.W;
        v.S = d.work;
        v.A = d.work + v.N;
        v.K = d.work + 2 * v.N;
        v.G = d.work + 3 * v.N;
        v.P = d.work + 4 * v.N;
        v.E = reinterpret_cast<uint32_t*>(d.work + ((5 * v.N + 3) & ~3ll));  // the block is 256-byte aligned
        for (long long q = threadIdx.x; q < v.N; q += VOL_NT) {
            const uint8_t x = d.X[q] != 0;
            v.S[q] = x;
            v.K[q] = d.C ? (uint8_t)(x && d.C[q] != 0) : 0;
        }
        __syncthreads();
        for (int i = 1; i <= d.r; ++i)
            for (int mode = 0; mode < 4; ++mode)
                vol_phase(v, i, mode, cnt, off, &s_flag);
        for (long long q = threadIdx.x; q < v.N; q += VOL_NT)
            d.X[q] = v.S[q];
        __syncthreads();
    }
}

namespace hasf_detail {

hipError_t launch_vol(const VolDesc* d_desc, int n, int* d_next, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(hasf_vol_kernel, dim3(grid), dim3(VOL_NT), 0, stream, d_desc, n, d_next);
    return hipGetLastError();
}

}  // namespace hasf_detail
