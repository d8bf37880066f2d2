/*
 * hasf_oracle3d.c -- 3D part of the CPU oracle (TEST INFRASTRUCTURE ONLY; the
 * same rules as hasf_oracle.c: only the tests, the smoke check and the
 * benchmark's CPU leg load it, and it shares nothing with the HIP library).
 *
 * The homotopic alternating sequential filter on 3D binary images with
 * 26-connected objects and a 6-connected background. The paper smooths 2D and
 * 3D objects (Sec. 1) and runs its distance transforms on 3D images
 * (Sec. 4.1); the operators are those of Sec. 2 with 3D balls and the 3D
 * topological numbers.
 *
 * Conventions (readings; the paper states the 2D case):
 *   - A volume is D x H x W bytes, voxel (z, y, x) at (z * H + y) * W + x,
 *     nonzero = object. Outside the box is background and never changes.
 *   - Neighbour b = 0..25 of a voxel is the offset (dz, dy, dx) in
 *     {-1, 0, 1}^3 without (0, 0, 0), in lexicographic order of (dz, dy, dx);
 *     a neighbourhood code has bit b set when neighbour b is object.
 *   - x is simple for (26,6) iff T26 = 1 and Tbar6 = 1: T26 is the number of
 *     26-components of the object voxels of the 26-neighbourhood (all of them
 *     are 26-adjacent to x); Tbar6 is the number of 6-components of the
 *     background voxels of the 18-neighbourhood that contain one of the six
 *     face neighbours of x.
 *   - Thinning and thickening: levels of increasing priority, and inside a
 *     level rounds of eight passes over the parity subfields
 *     (z mod 2, y mod 2, x mod 2) in lexicographic order, each pass acting
 *     on the state left by the previous one, until a round changes nothing.
 *     Two voxels of one subfield are never 26-adjacent.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O3_OK 0
#define O3_EINVAL (-1)
#define O3_ENOMEM (-2)
#define O3_INF 0xFFFFFFFFu

static int OFF[26][3];
static int off_ready = 0;

static void off_init(void)
{
    if (off_ready)
        return;
    int b = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dz && !dy && !dx)
                    continue;
                OFF[b][0] = dz;
                OFF[b][1] = dy;
                OFF[b][2] = dx;
                ++b;
            }
    off_ready = 1;
}

/* city-block and chessboard distances between neighbours a and b */
static int l1(int a, int b)
{
    return abs(OFF[a][0] - OFF[b][0]) + abs(OFF[a][1] - OFF[b][1]) + abs(OFF[a][2] - OFF[b][2]);
}

static int linf(int a, int b)
{
    int m = 0;
    for (int c = 0; c < 3; ++c) {
        const int d = abs(OFF[a][c] - OFF[b][c]);
        m = d > m ? d : m;
    }
    return m;
}

static int l1c(int a)
{
    return abs(OFF[a][0]) + abs(OFF[a][1]) + abs(OFF[a][2]);
}

/* components of the neighbour set `members` under 26- (adj = 26) or 6-adjacency
 * (adj = 6); with need_face, only those containing a face neighbour count */
static int o3_components(uint32_t members, int adj, int need_face)
{
    uint32_t seen = 0;
    int count = 0;
    for (int k = 0; k < 26; ++k) {
        if (!((members >> k) & 1u) || ((seen >> k) & 1u))
            continue;
        uint32_t comp = 1u << k, frontier = 1u << k;
        while (frontier) {
            uint32_t next = 0;
            for (int a = 0; a < 26; ++a) {
                if (!((frontier >> a) & 1u))
                    continue;
                for (int b = 0; b < 26; ++b) {
                    if (!((members >> b) & 1u) || ((comp >> b) & 1u))
                        continue;
                    if (adj == 26 ? linf(a, b) == 1 : l1(a, b) == 1)
                        next |= 1u << b;
                }
            }
            comp |= next;
            frontier = next;
        }
        seen |= comp;
        int face = 0;
        for (int a = 0; a < 26; ++a)
            if (((comp >> a) & 1u) && l1c(a) == 1)
                face = 1;
        count += need_face ? face : 1;
    }
    return count;
}

/* T26 and Tbar6 of the neighbourhood code */
int oracle3_topo_numbers(uint32_t code, int* T, int* Tbar)
{
    off_init();
    uint32_t n18 = 0;
    for (int b = 0; b < 26; ++b)
        if (l1c(b) <= 2)
            n18 |= 1u << b;
    *T = o3_components(code & 0x3FFFFFFu, 26, 0);
    *Tbar = o3_components(~code & n18, 6, 1);
    return O3_OK;
}

int oracle3_simple(uint32_t code)
{
    int T, Tb;
    oracle3_topo_numbers(code, &T, &Tb);
    return T == 1 && Tb == 1;
}

static uint32_t nbhd(const uint8_t* S, int D, int H, int W, int z, int y, int x)
{
    uint32_t code = 0;
    for (int b = 0; b < 26; ++b) {
        const int zz = z + OFF[b][0], yy = y + OFF[b][1], xx = x + OFF[b][2];
        if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W)
            continue;
        if (S[((size_t)zz * H + yy) * W + xx])
            code |= 1u << b;
    }
    return code;
}

/* ------------------------------------------------------------------------ */
/* Squared Euclidean distance to the nonzero voxels of F (and, with frame,  */
/* to every voxel outside the box), exact: the separable minimum along x,   */
/* then y, then z (Sec. 4.1 applies the transform to 3D images), each line  */
/* by a plain scan over the line.                                            */
/* ------------------------------------------------------------------------ */
static uint32_t sat_add(uint32_t a, uint32_t b)
{
    const uint64_t s = (uint64_t)a + b;
    return s >= O3_INF ? O3_INF : (uint32_t)s;
}

int oracle3_edt_sq(const uint8_t* F, int D, int H, int W, int frame, uint32_t* d2)
{
    if (D < 1 || H < 1 || W < 1)
        return O3_EINVAL;
    const int n = D > H ? (D > W ? D : W) : (H > W ? H : W);
    uint32_t* line = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    if (!line)
        return O3_ENOMEM;
    /* along x: squared distance to the nearest feature of the row */
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y) {
            const uint8_t* f = F + ((size_t)z * H + y) * W;
            uint32_t* o = d2 + ((size_t)z * H + y) * W;
            for (int x = 0; x < W; ++x) {
                uint32_t best = frame ? (uint32_t)((x + 1 < W - x ? x + 1 : W - x)) : O3_INF;
                if (best != O3_INF)
                    best *= best;
                for (int x2 = 0; x2 < W; ++x2)
                    if (f[x2]) {
                        const uint32_t d = (uint32_t)((x - x2) * (x - x2));
                        best = d < best ? d : best;
                    }
                o[x] = best;
            }
        }
    /* along y, then z: min over the line of (offset)^2 + previous value; with
     * the frame, the voxels just outside the box are features (value 0) */
    for (int pass = 0; pass < 2; ++pass) {
        const int len = pass == 0 ? H : D;
        for (int a = 0; a < (pass == 0 ? D : H); ++a)
            for (int x = 0; x < W; ++x) {
                size_t base, stride;
                if (pass == 0) {
                    base = (size_t)a * H * W + x;
                    stride = (size_t)W;
                } else {
                    base = (size_t)a * W + x;
                    stride = (size_t)H * W;
                }
                for (int t = 0; t < len; ++t)
                    line[t] = d2[base + t * stride];
                for (int t = 0; t < len; ++t) {
                    uint32_t best = O3_INF;
                    if (frame) {
                        const uint32_t e = (uint32_t)(t + 1 < len - t ? t + 1 : len - t);
                        best = e * e;
                    }
                    for (int t2 = 0; t2 < len; ++t2) {
                        const uint32_t v = sat_add(line[t2], (uint32_t)((t - t2) * (t - t2)));
                        best = v < best ? v : best;
                    }
                    d2[base + t * stride] = best;
                }
            }
    }
    free(line);
    return O3_OK;
}

/* ------------------------------------------------------------------------ */
/* Thinning H(S, B) (mode 0: delete simple voxels of S \ B) and thickening   */
/* *H(S, B) (mode 1: add simple voxels of B \ S), priority P, the schedule   */
/* above. Returns the number of changed voxels.                              */
/* ------------------------------------------------------------------------ */
static int cmp_u32(const void* a, const void* b)
{
    const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}

long oracle3_schedule(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P, int D, int H, int W)
{
    off_init();
    const size_t N = (size_t)D * H * W;
    for (size_t p = 0; p < N; ++p)
        S[p] = S[p] != 0;
    uint32_t* lv = (uint32_t*)malloc(sizeof(uint32_t) * (N ? N : 1));
    uint8_t* hit = (uint8_t*)malloc(N ? N : 1);
    if (!lv || !hit) {
        free(lv); free(hit);
        return O3_ENOMEM;
    }
    size_t nl = 0;
    for (size_t p = 0; p < N; ++p) {
        const int cand = mode == 0 ? (S[p] && !(B && B[p])) : (!S[p] && B && B[p]);
        if (cand && P[p] != O3_INF)
            lv[nl++] = P[p];
    }
    qsort(lv, nl, sizeof(uint32_t), cmp_u32);
    long changed = 0;
    for (size_t l = 0; l < nl; ++l) {
        if (l > 0 && lv[l] == lv[l - 1])
            continue;
        const uint32_t d = lv[l];
        for (;;) {
            int any = 0;
            for (int s = 0; s < 8; ++s) {
                const int pz = s >> 2, py = (s >> 1) & 1, px = s & 1;
                /* decide on the state before the pass, then apply */
                memset(hit, 0, N);
                for (int z = pz; z < D; z += 2)
                    for (int y = py; y < H; y += 2)
                        for (int x = px; x < W; x += 2) {
                            const size_t p = ((size_t)z * H + y) * W + x;
                            const int cand = mode == 0 ? (S[p] && !(B && B[p])) : (!S[p] && B && B[p]);
                            if (cand && P[p] <= d && oracle3_simple(nbhd(S, D, H, W, z, y, x)))
                                hit[p] = 1;
                        }
                for (size_t p = 0; p < N; ++p)
                    if (hit[p]) {
                        S[p] = (uint8_t)mode;
                        any = 1;
                        ++changed;
                    }
            }
            if (!any)
                break;
        }
    }
    free(lv);
    free(hit);
    return changed;
}

/* ------------------------------------------------------------------------ */
/* HC_i, HF_i and the filter (Sec. 2, eq. (i) and (ii) with W read as       */
/* eps_i(Z) u X; 3D Euclidean balls; priorities as in 2D: thinning by the   */
/* squared distance to the background and the outside, thickening by the    */
/* squared distance to the set being thickened).                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t *a, *b;
    uint32_t* P;
} work3_t;

static long hc3(uint8_t* X, const uint8_t* C, int D, int H, int W, int i, work3_t* w, uint8_t* stage)
{
    const size_t N = (size_t)D * H * W;
    const uint32_t r2 = (uint32_t)i * (uint32_t)i;
    uint8_t* K = w->a;
    uint8_t* Xs = w->b;
    long rc;
    for (size_t p = 0; p < N; ++p)
        K[p] = !X[p];
    if ((rc = oracle3_edt_sq(K, D, H, W, 1, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p) {
        K[p] = (X[p] && w->P[p] > r2) || (C && C[p]);
        Xs[p] = X[p];
    }
    if ((rc = oracle3_schedule(0, X, K, w->P, D, H, W)) < 0)
        return rc;
    if (stage)
        memcpy(stage, X, N);
    if ((rc = oracle3_edt_sq(X, D, H, W, 0, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        K[p] = w->P[p] <= r2 && Xs[p];
    if ((rc = oracle3_schedule(1, X, K, w->P, D, H, W)) < 0)
        return rc;
    if (stage)
        memcpy(stage + N, X, N);
    return 0;
}

static long hf3(uint8_t* X, int D, int H, int W, int i, work3_t* w, uint8_t* stage)
{
    const size_t N = (size_t)D * H * W;
    const uint32_t r2 = (uint32_t)i * (uint32_t)i;
    uint8_t* L = w->a;
    uint8_t* Xs = w->b;
    long rc;
    memcpy(Xs, X, N);
    if ((rc = oracle3_edt_sq(X, D, H, W, 0, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        L[p] = w->P[p] <= r2;
    if ((rc = oracle3_schedule(1, X, L, w->P, D, H, W)) < 0)
        return rc;
    if (stage)
        memcpy(stage, X, N);
    for (size_t p = 0; p < N; ++p)
        L[p] = !X[p];
    if ((rc = oracle3_edt_sq(L, D, H, W, 1, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        L[p] = (X[p] && w->P[p] > r2) || Xs[p];
    if ((rc = oracle3_schedule(0, X, L, w->P, D, H, W)) < 0)
        return rc;
    if (stage)
        memcpy(stage + N, X, N);
    return 0;
}

/* HASF of order r on a volume, constraint set C (C <- C n X; NULL = empty),
 * in place. stages: NULL or r * 4 * N bytes (per radius: after the cutting's
 * thinning, after the cutting, after the filling's thickening, after the
 * filling). */
long oracle3_hasf(uint8_t* X, const uint8_t* C, int D, int H, int W, int r, uint8_t* stages)
{
    if (D < 1 || H < 1 || W < 1 || r < 0)
        return O3_EINVAL;
    off_init();
    const size_t N = (size_t)D * H * W;
    for (size_t p = 0; p < N; ++p)
        X[p] = X[p] != 0;
    uint8_t* Cn = NULL;
    if (C) {
        Cn = (uint8_t*)malloc(N);
        if (!Cn)
            return O3_ENOMEM;
        for (size_t p = 0; p < N; ++p)
            Cn[p] = C[p] && X[p];
    }
    work3_t w;
    w.a = (uint8_t*)malloc(N);
    w.b = (uint8_t*)malloc(N);
    w.P = (uint32_t*)malloc(sizeof(uint32_t) * N);
    long rc = 0;
    if (!w.a || !w.b || !w.P)
        rc = O3_ENOMEM;
    for (int i = 1; i <= r && rc == 0; ++i) {
        uint8_t* st = stages ? stages + (size_t)(i - 1) * 4 * N : NULL;
        rc = hc3(X, Cn, D, H, W, i, &w, st);
        if (rc == 0)
            rc = hf3(X, D, H, W, i, &w, st ? st + 2 * N : NULL);
    }
    free(w.a); free(w.b); free(w.P); free(Cn);
    return rc < 0 ? rc : 0;
}
