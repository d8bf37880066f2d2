/*
 * hasf_oracle_wshed.c -- plain, single-threaded CPU oracle for the
 * topological watershed's lowering (grey-level W-thinning) on 2D grey-level
 * images. The paper places the topological watershed in the same class of
 * topology-based operators as its filter (Sec. 3.1) without defining it; the
 * reading taken here is the classical grey-level one, stated below.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code. It shares no code, header,
 * table or helper with the HIP library.
 *
 * Reading:
 *   - F is an H x W image of grey levels 0..255, row-major, one byte per
 *     pixel. For a level k the lower section is {p : F(p) < k}; lower
 *     sections are 4-connected (the background adjacency of the (8,4) pair
 *     of Sec. 2), their complements 8-connected. The plane outside the window
 *     never belongs to a lower section (it counts as higher than any level).
 *   - A pixel p is W-destructible when it has a lower neighbour and
 *     T-bar(p) = 1 for the binary image {q : F(q) >= F(p)} (object) against
 *     {q : F(q) < F(p)} (background) in its 8-neighbourhood: the background
 *     pixels of the neighbourhood that are 4-adjacent to p all lie in one
 *     4-component of the neighbourhood's background. Lowering such a p joins
 *     exactly one lower component and never merges two.
 *   - A W-destructible p is lowered to the largest grey level among its
 *     lower neighbours (8-neighbourhood): for every level between that value
 *     and F(p) its neighbourhood's lower section is the same, so p stays
 *     W-destructible all the way down.
 *   - Schedule: rounds of four passes over the 2x2 parity subfields
 *     (even,even) (even,odd) (odd,even) (odd,odd) of (row, column), each pass
 *     acting on the state before it, until a whole round changes nothing (no
 *     two pixels of one subfield are 8-adjacent, so a pass may lower its
 *     pixels in any order). Every lowering lowers a grey level, so it ends.
 *   - The result lowers no pixel that is not W-destructible, and every lower
 *     section's components stay in one-to-one correspondence with the input's
 *     (no merge, no new minimum); it is a fixed point of the lowering.
 */
#include <stdint.h>
#include <stddef.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

/* the topological numbers of hasf_oracle.c (the definitions of Sec. 2) */
int oracle_topo_numbers(int n, unsigned m, int* T, int* Tbar);

static const int WS_DY[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int WS_DX[8] = {1, 1, 0, -1, -1, -1, 0, 1};

/* Lowers the W-destructible pixels of F in place, to stability. Returns the
 * number of lowerings (>= 0) or ORACLE_EINVAL. */
long oracle_wshed(uint8_t* F, int H, int W)
{
    if (!F || H < 1 || W < 1)
        return ORACLE_EINVAL;
    long lowerings = 0;
    for (;;) {
        long round_changes = 0;
        for (int s = 0; s < 4; ++s) {
            const int si = s >> 1, sj = s & 1;
            for (int i = si; i < H; i += 2)
                for (int j = sj; j < W; j += 2) {
                    const int v = F[(size_t)i * W + j];
                    unsigned m = 0;  /* bit k: neighbour k is not lower (object) */
                    int delta = -1;  /* largest lower neighbour level */
                    for (int k = 0; k < 8; ++k) {
                        const int y = i + WS_DY[k], x = j + WS_DX[k];
                        if (y < 0 || y >= H || x < 0 || x >= W) {
                            m |= 1u << k;
                            continue;
                        }
                        const int f = F[(size_t)y * W + x];
                        if (f >= v)
                            m |= 1u << k;
                        else if (f > delta)
                            delta = f;
                    }
                    if (delta < 0)
                        continue;
                    int T, Tbar;
                    oracle_topo_numbers(8, m, &T, &Tbar);
                    if (Tbar == 1) {
                        F[(size_t)i * W + j] = (uint8_t)delta;
                        ++round_changes;
                    }
                }
        }
        lowerings += round_changes;
        if (round_changes == 0)
            break;
    }
    return lowerings;
}
