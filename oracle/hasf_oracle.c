/*
 * hasf_oracle.c -- plain, slow, single-threaded CPU oracle for the homotopic
 * alternating sequential filter (HASF) of Mahmoudi & Akil, "Real Time
 * Topological Image Smoothing On Shared Memory Parallel Machines"
 * (arXiv:1603.09337).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code. It shares no code, header,
 * table or helper with the HIP library; it is written from the paper's
 * definitions so that the GPU path can be checked against it.
 *
 * Conventions used throughout (the paper leaves them open; each is a stated
 * reading):
 *   - Images are H x W, row-major, one byte per pixel, nonzero = object.
 *     Coordinates are (row i, column j); the plane outside the window is
 *     background and never changes (X is a finite subset of Z^2, Sec. 2).
 *   - Neighbour k of a pixel, k = 0..7, is the direction
 *     E(0,+1) NE(-1,+1) N(-1,0) NW(-1,-1) W(0,-1) SW(+1,-1) S(+1,0) SE(+1,+1);
 *     a neighbourhood code m has bit k set when neighbour k is object.
 *   - Thinning and thickening follow one deterministic schedule: distance
 *     levels in increasing order, and inside a level, rounds of four passes
 *     over the 2x2 parity subfields (even,even) (even,odd) (odd,even)
 *     (odd,odd) of (row, column), each pass acting on the state before it,
 *     until a whole round changes nothing.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

static const int NB_DY[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int NB_DX[8] = {1, 1, 0, -1, -1, -1, 0, 1};

/* ------------------------------------------------------------------------ */
/* Topological numbers and the simple-point table (Sec. 2, the definitions   */
/* of n-adjacency, n-components, C_n[x,X], T and T-bar, and the local        */
/* characterisation: x is simple iff T = 1 and T-bar = 1).                   */
/* ------------------------------------------------------------------------ */

/* Two ring points are n-adjacent: 4 -> city-block distance 1, 8 -> chessboard 1. */
static int ring_adjacent(int k, int l, int n)
{
    int dy = abs(NB_DY[k] - NB_DY[l]);
    int dx = abs(NB_DX[k] - NB_DX[l]);
    if (dy == 0 && dx == 0)
        return 0;
    if (n == 4)
        return dy + dx == 1;
    return dy <= 1 && dx <= 1;
}

/* Ring point k is n-adjacent to the centre. */
static int centre_adjacent(int k, int n)
{
    return n == 8 ? 1 : (NB_DY[k] == 0 || NB_DX[k] == 0);
}

/* Number of n-components of the ring subset `members` (bit k = point k) that
 * are n-adjacent to the centre: #C_n[x, members]. */
static int count_components(unsigned members, int n)
{
    unsigned seen = 0;
    int count = 0;
    for (int k = 0; k < 8; ++k) {
        if (!((members >> k) & 1u) || ((seen >> k) & 1u))
            continue;
        /* flood fill the component that contains k */
        unsigned comp = 1u << k, frontier = 1u << k;
        while (frontier) {
            unsigned next = 0;
            for (int a = 0; a < 8; ++a) {
                if (!((frontier >> a) & 1u))
                    continue;
                for (int b = 0; b < 8; ++b)
                    if (((members >> b) & 1u) && !((comp >> b) & 1u) && ring_adjacent(a, b, n))
                        next |= 1u << b;
            }
            comp |= next;
            frontier = next;
        }
        seen |= comp;
        int touches = 0;
        for (int a = 0; a < 8; ++a)
            if (((comp >> a) & 1u) && centre_adjacent(a, n))
                touches = 1;
        count += touches;
    }
    return count;
}

/* T(x, X) for object adjacency n, T-bar(x, X) for the complementary adjacency. */
int oracle_topo_numbers(int n, unsigned m, int* T, int* Tbar)
{
    if (n != 8 && n != 4)
        return ORACLE_EINVAL;
    int nbar = n == 8 ? 4 : 8;
    *T = count_components(m & 0xFFu, n);
    *Tbar = count_components((~m) & 0xFFu, nbar);
    return ORACLE_OK;
}

/* lut[m] = 1 iff a point with neighbourhood code m is simple for (n, n-bar). */
int oracle_simple_lut(int n, uint8_t* lut)
{
    if (n != 8 && n != 4)
        return ORACLE_EINVAL;
    for (unsigned m = 0; m < 256; ++m) {
        int T, Tb;
        oracle_topo_numbers(n, m, &T, &Tb);
        lut[m] = (uint8_t)(T == 1 && Tb == 1);
    }
    return ORACLE_OK;
}

static unsigned nbhd_code(const uint8_t* S, int H, int W, int i, int j)
{
    unsigned m = 0;
    for (int k = 0; k < 8; ++k) {
        int y = i + NB_DY[k], x = j + NB_DX[k];
        if (y >= 0 && y < H && x >= 0 && x < W && S[(size_t)y * W + x])
            m |= 1u << k;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Squared Euclidean distance transform (Sec. 4.1).                          */
/* ------------------------------------------------------------------------ */

/* Definition: d2(p) = min over feature pixels q of |p - q|^2, where the
 * features are the nonzero pixels of `feat` and, when `frame` is set, every
 * pixel outside the window. Computed directly, with the minimum regrouped by
 * column: min_k [ (j - k)^2 + min_r { (i - r)^2 : q = (r, k) feature } ].
 * O(H*W*(H+W)). An empty feature set (frame unset) gives UINT32_MAX. */
int oracle_edt_sq_direct(const uint8_t* feat, int H, int W, int frame, uint32_t* d2)
{
    if (H < 1 || W < 1)
        return ORACLE_EINVAL;
    /* gcol[i*W + k] = min_r |i - r| over features in column k (-1: none) */
    int64_t* gcol = (int64_t*)malloc(sizeof(int64_t) * (size_t)H * W);
    if (!gcol)
        return ORACLE_ENOMEM;
    for (int i = 0; i < H; ++i)
        for (int k = 0; k < W; ++k) {
            int64_t best = -1;
            for (int r = 0; r < H; ++r)
                if (feat[(size_t)r * W + k]) {
                    int64_t d = r > i ? r - i : i - r;
                    if (best < 0 || d < best)
                        best = d;
                }
            if (frame) { /* rows -1 and H are outside the window */
                int64_t d = i + 1 < H - i ? i + 1 : H - i;
                if (best < 0 || d < best)
                    best = d;
            }
            gcol[(size_t)i * W + k] = best;
        }
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            int64_t best = -1;
            for (int k = 0; k < W; ++k) {
                int64_t g = gcol[(size_t)i * W + k];
                if (g < 0)
                    continue;
                int64_t v = (int64_t)(j - k) * (j - k) + g * g;
                if (best < 0 || v < best)
                    best = v;
            }
            if (frame) { /* columns -1 and W, any row: nearest is the same row */
                int64_t dj = j + 1 < W - j ? j + 1 : W - j;
                if (best < 0 || dj * dj < best)
                    best = dj * dj;
            }
            d2[(size_t)i * W + j] = best < 0 ? UINT32_MAX : (uint32_t)best;
        }
    free(gcol);
    return ORACLE_OK;
}

/* Meijster's two-phase exact transform as the paper describes it (Alg. 1 and
 * Alg. 2 of Sec. 4.1, with the readings: the top-down scan adds one to the
 * value of the row above; the envelope is popped while the last parabola is
 * worse than the new one at the start of its region; Sep(i,u) =
 * (u^2 - i^2 + g(u)^2 - g(i)^2) div (2(u - i)); infinity = h + w).
 * Bit-exact to oracle_edt_sq_direct (the tests pin it there); used by the
 * filter only because the direct form is too slow at large sizes. */
static int edt_meijster_core(const uint8_t* F, int h, int w, uint32_t* out, int* any_feature)
{
    const int64_t inf = (int64_t)h + w;
    int64_t* g = (int64_t*)malloc(sizeof(int64_t) * (size_t)h * w);
    int* s = (int*)malloc(sizeof(int) * (size_t)w);
    int* t = (int*)malloc(sizeof(int) * (size_t)w);
    if (!g || !s || !t) {
        free(g); free(s); free(t);
        return ORACLE_ENOMEM;
    }
    int any = 0;
    /* phase 1: per column, distance to the nearest feature in that column */
    for (int y = 0; y < w; ++y) {
        g[y] = F[y] ? 0 : inf;
        any |= F[y] != 0;
        for (int x = 1; x < h; ++x) {
            if (F[(size_t)x * w + y]) {
                g[(size_t)x * w + y] = 0;
                any = 1;
            } else {
                g[(size_t)x * w + y] = g[(size_t)(x - 1) * w + y] + 1;
            }
        }
        for (int x = h - 2; x >= 0; --x)
            if (g[(size_t)(x + 1) * w + y] < g[(size_t)x * w + y])
                g[(size_t)x * w + y] = g[(size_t)(x + 1) * w + y] + 1;
    }
    /* phase 2: per row, lower envelope of the parabolas f(u, i) = (u-i)^2 + g(i)^2 */
    for (int x = 0; x < h; ++x) {
        const int64_t* gr = g + (size_t)x * w;
#define F_AT(uu, ii) ((int64_t)((uu) - (ii)) * ((uu) - (ii)) + gr[ii] * gr[ii])
        int q = 0;
        s[0] = 0;
        t[0] = 0;
        for (int u = 1; u < w; ++u) {
            while (q >= 0 && F_AT(t[q], s[q]) > F_AT(t[q], u))
                --q;
            if (q < 0) {
                q = 0;
                s[0] = u;
            } else {
                int64_t i0 = s[q];
                int64_t num = (int64_t)u * u - i0 * i0 + gr[u] * gr[u] - gr[i0] * gr[i0];
                int64_t den = 2 * ((int64_t)u - i0);
                int64_t sep = num >= 0 ? num / den : -((-num + den - 1) / den);
                int64_t wv = sep + 1;
                if (wv < w) {
                    ++q;
                    s[q] = u;
                    t[q] = (int)wv;
                }
            }
        }
        for (int u = w - 1; u >= 0; --u) {
            int64_t v = F_AT(u, s[q]);
            out[(size_t)x * w + u] = (uint32_t)v;
            if (u == t[q])
                --q;
        }
#undef F_AT
    }
    free(g); free(s); free(t);
    *any_feature = any;
    return ORACLE_OK;
}

int oracle_edt_sq(const uint8_t* feat, int H, int W, int frame, uint32_t* d2)
{
    if (H < 1 || W < 1)
        return ORACLE_EINVAL;
    int any = 0, rc;
    if (!frame) {
        rc = edt_meijster_core(feat, H, W, d2, &any);
        if (rc)
            return rc;
    } else {
        /* pad by one pixel of feature: the nearest point outside the window
         * always lies on that ring */
        int h = H + 2, w = W + 2;
        uint8_t* F = (uint8_t*)malloc((size_t)h * w);
        uint32_t* o = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)h * w);
        if (!F || !o) {
            free(F); free(o);
            return ORACLE_ENOMEM;
        }
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j)
                F[(size_t)i * w + j] = (i == 0 || j == 0 || i == h - 1 || j == w - 1)
                                           ? 1 : (feat[(size_t)(i - 1) * W + (j - 1)] != 0);
        rc = edt_meijster_core(F, h, w, o, &any);
        if (!rc)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j)
                    d2[(size_t)i * W + j] = o[(size_t)(i + 1) * w + (j + 1)];
        free(F); free(o);
        if (rc)
            return rc;
    }
    if (!any)
        for (size_t p = 0; p < (size_t)H * W; ++p)
            d2[p] = UINT32_MAX;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Constrained thinning H(S, K) and thickening *H(S, V) (Sec. 2): simple    */
/* points are deleted (added) in increasing order of a precomputed distance */
/* map P; a point of level <= d stays eligible at level d.                  */
/* ------------------------------------------------------------------------ */

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y);
}

/* Sorted distinct values of P over the pixels where sel != 0. */
static uint32_t* distinct_levels(const uint32_t* P, const uint8_t* sel, size_t N, size_t* nlev)
{
    size_t n = 0;
    for (size_t p = 0; p < N; ++p)
        n += sel[p] != 0;
    uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!v)
        return NULL;
    n = 0;
    for (size_t p = 0; p < N; ++p)
        if (sel[p])
            v[n++] = P[p];
    qsort(v, n, sizeof(uint32_t), cmp_u32);
    size_t u = 0;
    for (size_t k = 0; k < n; ++k)
        if (u == 0 || v[k] != v[u - 1])
            v[u++] = v[k];
    *nlev = u;
    return v;
}

/* mode 0: thin S, eligible = S & !B; mode 1: thicken S, eligible = !S & B.
 * B is the constraint set K (thin) or the limit set V (thicken); NULL = empty.
 * Returns the number of rounds run, or a negative error. */
static long subfield_schedule(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P,
                              int H, int W, const uint8_t* lut)
{
    const size_t N = (size_t)H * W;
    uint8_t* cand = (uint8_t*)malloc(N);
    size_t* D = (size_t*)malloc(sizeof(size_t) * (N / 4 + 4));
    if (!cand || !D) {
        free(cand); free(D);
        return ORACLE_ENOMEM;
    }
    for (size_t p = 0; p < N; ++p) {
        int b = B ? B[p] != 0 : 0;
        cand[p] = mode == 0 ? (S[p] && !b) : (!S[p] && b);
    }
    size_t nlev = 0;
    uint32_t* lev = distinct_levels(P, cand, N, &nlev);
    if (!lev) {
        free(cand); free(D);
        return ORACLE_ENOMEM;
    }
    long rounds = 0;
    const long cap = (long)N + 1;
    for (size_t l = 0; l < nlev; ++l) {
        const uint32_t d = lev[l];
        long rounds_here = 0;
        for (;;) {
            int any = 0;
            for (int s = 0; s < 4; ++s) {
                const int si = s >> 1, sj = s & 1;
                size_t nd = 0;
                for (int i = si; i < H; i += 2)
                    for (int j = sj; j < W; j += 2) {
                        size_t p = (size_t)i * W + j;
                        int b = B ? B[p] != 0 : 0;
                        int elig = mode == 0 ? (S[p] && !b) : (!S[p] && b);
                        if (elig && P[p] <= d && lut[nbhd_code(S, H, W, i, j)])
                            D[nd++] = p;
                    }
                for (size_t k = 0; k < nd; ++k)
                    S[D[k]] = (uint8_t)(mode == 1);
                any |= nd > 0;
            }
            ++rounds;
            if (!any)
                break;
            if (++rounds_here > cap) { /* cannot happen: each round changes >= 1 pixel */
                free(cand); free(D); free(lev);
                return -6;
            }
        }
    }
    free(cand); free(D); free(lev);
    return rounds;
}

static uint8_t g_lut84[256], g_lut48[256];
static int g_lut_ready = 0;

static void luts_init(void)
{
    if (!g_lut_ready) {
        oracle_simple_lut(8, g_lut84);
        oracle_simple_lut(4, g_lut48);
        g_lut_ready = 1;
    }
}

static const uint8_t* lut84(void)
{
    luts_init();
    return g_lut84;
}

/* simple points for the pair (n, n-bar) = (8, 4) or (4, 8) (Sec. 2) */
static const uint8_t* lut_for(int n)
{
    luts_init();
    return n == 4 ? g_lut48 : g_lut84;
}

/* Thinning with an explicit priority map (for tests). */
long oracle_thin_p(uint8_t* S, const uint8_t* K, const uint32_t* P, int H, int W)
{
    return subfield_schedule(0, S, K, P, H, W, lut84());
}

long oracle_thicken_p(uint8_t* S, const uint8_t* V, const uint32_t* P, int H, int W)
{
    return subfield_schedule(1, S, V, P, H, W, lut84());
}

/* Thinning with a caller-supplied simple-point table (planted-mistake tests). */
long oracle_thin_p_lut(uint8_t* S, const uint8_t* K, const uint32_t* P, int H, int W,
                       const uint8_t* lut)
{
    return subfield_schedule(0, S, K, P, H, W, lut);
}

static void normalise(uint8_t* X, size_t N)
{
    for (size_t p = 0; p < N; ++p)
        X[p] = X[p] != 0;
}

/* H(X, K) for the pair (n, n-bar) (n = 8: (8,4); n = 4: (4,8)): priority =
 * squared distance to the background, the outside of the window included. */
long oracle_homotopic_thin_n(uint8_t* X, const uint8_t* K, int H, int W, int n)
{
    if (H < 1 || W < 1 || (n != 8 && n != 4))
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(X, N);
    uint8_t* bg = (uint8_t*)malloc(N);
    uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * N);
    if (!bg || !P) {
        free(bg); free(P);
        return ORACLE_ENOMEM;
    }
    for (size_t p = 0; p < N; ++p)
        bg[p] = !X[p];
    long rc = oracle_edt_sq(bg, H, W, 1, P);
    if (rc == 0)
        rc = subfield_schedule(0, X, K, P, H, W, lut_for(n));
    free(bg); free(P);
    return rc;
}

long oracle_homotopic_thin(uint8_t* X, const uint8_t* K, int H, int W)
{
    return oracle_homotopic_thin_n(X, K, H, W, 8);
}

/* *H(Y, V) for the pair (n, n-bar): priority = squared distance to Y. */
long oracle_homotopic_thicken_n(uint8_t* Y, const uint8_t* V, int H, int W, int n)
{
    if (H < 1 || W < 1 || (n != 8 && n != 4))
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(Y, N);
    uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * N);
    if (!P)
        return ORACLE_ENOMEM;
    long rc = oracle_edt_sq(Y, H, W, 0, P);
    if (rc == 0)
        rc = subfield_schedule(1, Y, V, P, H, W, lut_for(n));
    free(P);
    return rc;
}

long oracle_homotopic_thicken(uint8_t* Y, const uint8_t* V, int H, int W)
{
    return oracle_homotopic_thicken_n(Y, V, H, W, 8);
}

/* ------------------------------------------------------------------------ */
/* Homotopic cutting, filling and the alternating sequential filter          */
/* (Sec. 2, eq. (i), eq. (ii) with W read as eps_n(Z) u X, and the           */
/* composition HASF = HF_r o HC_r o ... o HF_1 o HC_1).                      */
/* ------------------------------------------------------------------------ */

typedef long (*sched_fn)(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P, int H, int W,
                         const uint8_t* lut);

static long sched_subfield(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P, int H, int W,
                           const uint8_t* lut)
{
    return subfield_schedule(mode, S, B, P, H, W, lut);
}

static long queue_schedule(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P, int H, int W,
                           const uint8_t* lut);

typedef struct {
    uint8_t* a;          /* N bytes */
    uint8_t* b;          /* N bytes */
    uint32_t* P;         /* N words */
    sched_fn run;        /* thinning / thickening schedule */
    const uint8_t* lut;  /* simple-point table of the connectivity pair */
} work_t;

/* HC_i with constraint C (C subset of X, NULL = empty). stage: 2 x N bytes or NULL. */
static long hc(uint8_t* X, const uint8_t* C, int H, int W, int i, work_t* w, uint8_t* stage)
{
    const size_t N = (size_t)H * W;
    const uint32_t r2 = (uint32_t)i * (uint32_t)i;
    uint8_t* K = w->a;
    uint8_t* Xs = w->b;
    long rc;
    for (size_t p = 0; p < N; ++p)
        K[p] = !X[p];
    if ((rc = oracle_edt_sq(K, H, W, 1, w->P)))
        return rc;
    /* K = eps_i(X) u C ; eps_i(X) = { p in X : d2(p, complement) > i^2 } */
    for (size_t p = 0; p < N; ++p) {
        K[p] = (X[p] && w->P[p] > r2) || (C && C[p]);
        Xs[p] = X[p];
    }
    if ((rc = w->run(0, X, K, w->P, H, W, w->lut)) < 0)
        return rc;
    if (stage)
        memcpy(stage, X, N);
    /* V = delta_i(Y) n X, priority = d2(., Y) */
    if ((rc = oracle_edt_sq(X, H, W, 0, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        K[p] = w->P[p] <= r2 && Xs[p];
    if ((rc = w->run(1, X, K, w->P, H, W, w->lut)) < 0)
        return rc;
    if (stage)
        memcpy(stage + N, X, N);
    return 0;
}

/* HF_i with background constraint D (D in the complement of X, NULL = empty). */
static long hf(uint8_t* X, const uint8_t* D, int H, int W, int i, work_t* w, uint8_t* stage)
{
    const size_t N = (size_t)H * W;
    const uint32_t r2 = (uint32_t)i * (uint32_t)i;
    uint8_t* L = w->a;
    uint8_t* Xs = w->b;
    long rc;
    memcpy(Xs, X, N);
    /* L = delta_i(X) n complement(D) (inside the window), priority = d2(., X) */
    if ((rc = oracle_edt_sq(X, H, W, 0, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        L[p] = w->P[p] <= r2 && !(D && D[p]);
    if ((rc = w->run(1, X, L, w->P, H, W, w->lut)) < 0)
        return rc;
    if (stage)
        memcpy(stage, X, N);
    /* W = eps_i(Z) u X, priority = d2(., complement of Z) */
    for (size_t p = 0; p < N; ++p)
        L[p] = !X[p];
    if ((rc = oracle_edt_sq(L, H, W, 1, w->P)))
        return rc;
    for (size_t p = 0; p < N; ++p)
        L[p] = (X[p] && w->P[p] > r2) || Xs[p];
    if ((rc = w->run(0, X, L, w->P, H, W, w->lut)) < 0)
        return rc;
    if (stage)
        memcpy(stage + N, X, N);
    return 0;
}

static int work_alloc(work_t* w, size_t N, sched_fn run)
{
    w->run = run;
    w->lut = lut84();
    w->a = (uint8_t*)malloc(N);
    w->b = (uint8_t*)malloc(N);
    w->P = (uint32_t*)malloc(sizeof(uint32_t) * N);
    if (!w->a || !w->b || !w->P) {
        free(w->a); free(w->b); free(w->P);
        return ORACLE_ENOMEM;
    }
    return 0;
}

static void work_free(work_t* w)
{
    free(w->a); free(w->b); free(w->P);
}

/* One homotopic cutting (with C) at radius i, in place. */
long oracle_hc(uint8_t* X, const uint8_t* C, int H, int W, int i)
{
    if (H < 1 || W < 1 || i < 0)
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(X, N);
    uint8_t* Cn = NULL;
    if (C) {
        Cn = (uint8_t*)malloc(N);
        if (!Cn)
            return ORACLE_ENOMEM;
        for (size_t p = 0; p < N; ++p)
            Cn[p] = C[p] && X[p];
    }
    work_t w;
    long rc = work_alloc(&w, N, sched_subfield);
    if (rc) {
        free(Cn);
        return rc;
    }
    rc = hc(X, Cn, H, W, i, &w, NULL);
    work_free(&w);
    free(Cn);
    return rc < 0 ? rc : 0;
}

/* One homotopic filling at radius i, in place. */
long oracle_hf(uint8_t* X, int H, int W, int i)
{
    if (H < 1 || W < 1 || i < 0)
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(X, N);
    work_t w;
    long rc = work_alloc(&w, N, sched_subfield);
    if (rc)
        return rc;
    rc = hf(X, NULL, H, W, i, &w, NULL);
    work_free(&w);
    return rc < 0 ? rc : 0;
}

/* order 0: HF_i o HC_i at every radius (the formula of Sec. 2, cutting
 * first); order 1: the dual sequence HC_i o HF_i (filling first). */
static long hasf_core(uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W, int r, int n, int order,
                      uint8_t* stages, sched_fn run)
{
    if (H < 1 || W < 1 || r < 0 || (n != 8 && n != 4) || (order != 0 && order != 1))
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(X, N);
    /* C <- C n X and D <- D \ X (Sec. 2: C is a subset of X, D of its complement) */
    uint8_t* Cn = NULL;
    uint8_t* Dn = NULL;
    if (C || D) {
        Cn = (uint8_t*)malloc(N);
        Dn = (uint8_t*)malloc(N);
        if (!Cn || !Dn) {
            free(Cn); free(Dn);
            return ORACLE_ENOMEM;
        }
        for (size_t p = 0; p < N; ++p) {
            Cn[p] = C && C[p] && X[p];
            Dn[p] = D && D[p] && !X[p];
        }
    }
    work_t w;
    long rc = work_alloc(&w, N, run);
    if (rc) {
        free(Cn); free(Dn);
        return rc;
    }
    w.lut = lut_for(n);
    for (int i = 1; i <= r && rc == 0; ++i) {
        uint8_t* st = stages ? stages + (size_t)(i - 1) * 4 * N : NULL;
        if (order == 0) {
            rc = hc(X, C ? Cn : NULL, H, W, i, &w, st);
            if (rc == 0)
                rc = hf(X, D ? Dn : NULL, H, W, i, &w, st ? st + 2 * N : NULL);
        } else {
            rc = hf(X, D ? Dn : NULL, H, W, i, &w, st);
            if (rc == 0)
                rc = hc(X, C ? Cn : NULL, H, W, i, &w, st ? st + 2 * N : NULL);
        }
    }
    work_free(&w);
    free(Cn); free(Dn);
    return rc;
}

/* HASF of order r with constraint set C (C <- C n X; NULL = empty), in place.
 * stages (NULL or r*4*H*W bytes) receives, for each radius i, the state after
 * the cutting's thinning, after the cutting, after the filling's thickening
 * and after the filling. */
long oracle_hasf(uint8_t* X, const uint8_t* C, int H, int W, int r, uint8_t* stages)
{
    return hasf_core(X, C, NULL, H, W, r, 8, 0, stages, sched_subfield);
}

/* HASF^{C,D} of order r for the connectivity pair (n, n-bar), n = 8: (8,4),
 * n = 4: (4,8) (Sec. 2): the cutting keeps C (C <- C n X), the filling never
 * adds a point of D (D <- D \ X), so D stays background. NULL = empty. */
long oracle_hasf_cd(uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W, int r, int n, uint8_t* stages)
{
    return hasf_core(X, C, D, H, W, r, n, 0, stages, sched_subfield);
}

/* As oracle_hasf_cd, in the given order: 0 = HF_i o HC_i at every radius (the
 * formula), 1 = the dual HC_i o HF_i (filling first). stages then holds, per
 * radius, the four states in the order they are produced. */
long oracle_hasf_order(uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W, int r, int n, int order,
                       uint8_t* stages)
{
    return hasf_core(X, C, D, H, W, r, n, order, stages, sched_subfield);
}

/* "r = infinity" (the column of Tab. 1, which the paper does not define):
 * radii i = 1, 2, ... as in oracle_hasf_order, stopping after the first
 * radius whose cutting and filling leave X unchanged, and at the latest after
 * radius r_max (r_max <= 0: the saturation radius, the least i with
 * i^2 >= (H-1)^2 + (W-1)^2; from there on every threshold and every level
 * test of a radius holds for all pixels, so every larger radius applies the
 * same operator). C <- C n X and D <- D \ X from the input, as for a finite
 * radius. *r_used receives the last radius applied (at least 1). */
long oracle_hasf_inf(uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W, int n, int order, int r_max,
                     int* r_used)
{
    if (H < 1 || W < 1 || (n != 8 && n != 4) || (order != 0 && order != 1) || !r_used)
        return ORACLE_EINVAL;
    const size_t N = (size_t)H * W;
    normalise(X, N);
    int cap = r_max;
    if (cap <= 0) {
        const long long far = (long long)(H - 1) * (H - 1) + (long long)(W - 1) * (W - 1);
        cap = 1;
        while ((long long)cap * cap < far)
            ++cap;
    }
    uint8_t* Cn = (uint8_t*)malloc(N);
    uint8_t* Dn = (uint8_t*)malloc(N);
    uint8_t* prev = (uint8_t*)malloc(N);
    if (!Cn || !Dn || !prev) {
        free(Cn); free(Dn); free(prev);
        return ORACLE_ENOMEM;
    }
    for (size_t p = 0; p < N; ++p) {
        Cn[p] = C && C[p] && X[p];
        Dn[p] = D && D[p] && !X[p];
    }
    work_t w;
    long rc = work_alloc(&w, N, sched_subfield);
    if (rc) {
        free(Cn); free(Dn); free(prev);
        return rc;
    }
    w.lut = lut_for(n);
    *r_used = 0;
    for (int i = 1; i <= cap && rc == 0; ++i) {
        memcpy(prev, X, N);
        if (order == 0) {
            rc = hc(X, C ? Cn : NULL, H, W, i, &w, NULL);
            if (rc == 0)
                rc = hf(X, D ? Dn : NULL, H, W, i, &w, NULL);
        } else {
            rc = hf(X, D ? Dn : NULL, H, W, i, &w, NULL);
            if (rc == 0)
                rc = hc(X, C ? Cn : NULL, H, W, i, &w, NULL);
        }
        *r_used = i;
        if (rc == 0 && memcmp(prev, X, N) == 0)
            break;
    }
    work_free(&w);
    free(Cn); free(Dn); free(prev);
    return rc < 0 ? rc : 0;
}

/* The same filter with the queue-ordered schedule below. */
long oracle_hasf_queue(uint8_t* X, const uint8_t* C, int H, int W, int r)
{
    return hasf_core(X, C, NULL, H, W, r, 8, 0, NULL, queue_schedule);
}

/* ------------------------------------------------------------------------ */
/* Queue-ordered variant ("oracle B"): the same operators with the deletion  */
/* order of a priority queue keyed by (P, arrival), in the spirit of the     */
/* worklist thinning of Sec. 4.2 (a deleted point sends its 8 neighbours     */
/* back for re-testing). Its result may differ from the subfield schedule    */
/* in pixels; the tests only check it for invariants.                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t key;
    uint64_t seq;
    size_t p;
} hnode;

static int hless(const hnode* a, const hnode* b)
{
    return a->key < b->key || (a->key == b->key && a->seq < b->seq);
}

static void hpush(hnode* h, size_t* n, hnode v)
{
    size_t i = (*n)++;
    h[i] = v;
    while (i > 0) {
        size_t par = (i - 1) / 2;
        if (!hless(&h[i], &h[par]))
            break;
        hnode t = h[i]; h[i] = h[par]; h[par] = t;
        i = par;
    }
}

static hnode hpop(hnode* h, size_t* n)
{
    hnode top = h[0];
    h[0] = h[--(*n)];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && hless(&h[l], &h[m])) m = l;
        if (r < *n && hless(&h[r], &h[m])) m = r;
        if (m == i)
            break;
        hnode t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

static long queue_schedule(int mode, uint8_t* S, const uint8_t* B, const uint32_t* P, int H, int W,
                           const uint8_t* lut)
{
    const size_t N = (size_t)H * W;
    /* a pixel is queued at most once at a time: heap size <= N */
    hnode* heap = (hnode*)malloc(sizeof(hnode) * (N + 1));
    uint8_t* inq = (uint8_t*)calloc(N, 1);
    if (!heap || !inq) {
        free(heap); free(inq);
        return ORACLE_ENOMEM;
    }
    size_t n = 0;
    uint64_t seq = 0;
#define ELIG(p) (mode == 0 ? (S[p] && !(B && B[p])) : (!S[p] && (B && B[p])))
    for (size_t p = 0; p < N; ++p)
        if (ELIG(p)) {
            hnode v = {P[p], seq++, p};
            hpush(heap, &n, v);
            inq[p] = 1;
        }
    long changes = 0;
    while (n) {
        hnode v = hpop(heap, &n);
        size_t p = v.p;
        inq[p] = 0;
        int i = (int)(p / W), j = (int)(p % W);
        if (!ELIG(p) || !lut[nbhd_code(S, H, W, i, j)])
            continue;
        S[p] = (uint8_t)(mode == 1);
        ++changes;
        for (int k = 0; k < 8; ++k) {
            int y = i + NB_DY[k], x = j + NB_DX[k];
            if (y < 0 || y >= H || x < 0 || x >= W)
                continue;
            size_t q = (size_t)y * W + x;
            if (!inq[q] && ELIG(q)) {
                hnode u = {P[q], seq++, q};
                hpush(heap, &n, u);
                inq[q] = 1;
            }
        }
    }
#undef ELIG
    free(heap); free(inq);
    return changes;
}

long oracle_thin_queue_p(uint8_t* S, const uint8_t* K, const uint32_t* P, int H, int W)
{
    return queue_schedule(0, S, K, P, H, W, lut84());
}

long oracle_thicken_queue_p(uint8_t* S, const uint8_t* V, const uint32_t* P, int H, int W)
{
    return queue_schedule(1, S, V, P, H, W, lut84());
}
