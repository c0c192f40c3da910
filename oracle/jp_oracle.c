/*
 * Serial CPU oracle for the Jones-Plassmann (JP) independent-set colouring of
 * Sec. 2.2, Algorithm 3 -- TEST INFRASTRUCTURE ONLY.  Nothing in the product library
 * calls, links or includes this file; it shares no code with the GPU path.
 *
 * What it computes:
 *
 *   W = V, c = 1
 *   while W is not empty:                          one round, colour c
 *     for v in W:  r(v) = priority of v in round c (a fresh random number)
 *     S = { v in W : r(v) > r(w) for every neighbour w in W, w != v }
 *     colour every v in S with c;  W = W - S;  c = c + 1
 *
 * Readings taken where the paper leaves freedom:
 *   - only neighbours still in W take part in the comparison: r is drawn for W only,
 *     and coloured vertices have left the shrinking graph;
 *   - a tie r(v) == r(w) would keep both out of S (the printed test rejects v when
 *     r(v) <= r(w)), but with the generator below it cannot occur: k -> seed + k*gamma
 *     is a bijection (gamma is odd) and so is the output function, so distinct
 *     vertices of one round get distinct priorities, the priority maximum of W always
 *     joins S, and the loop ends within |V| rounds;
 *   - self-loops are ignored (a vertex never blocks itself);
 *   - the random numbers are a counter-based generator, so the result is a function
 *     of (graph, seed): r(v) in round c is output number k = c * 2^32 + v of
 *     SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) seeded with `seed`, i.e.
 *     mix(seed + k * 0x9E3779B97F4A7C15) with the generator's published output
 *     function, compared as unsigned 64-bit integers;
 *   - colours are exported 0-based (c - 1); ncolors = number of rounds.
 */
#include <stdint.h>
#include <stdlib.h>

/* Output number k (k >= 1) of SplitMix64 seeded with `seed`. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_jp_priority(uint64_t seed, int32_t round, int32_t v)
{
    return oracle_splitmix64(seed, ((uint64_t)(uint32_t)round << 32) + (uint64_t)(uint32_t)v);
}

/* Per-round statistics (any pointer may be NULL): wsize[r] = |W_r|, arcs[r] = sum of
 * row lengths over W_r.  Returns 0, -1 on allocation failure, -2 if a colidx entry
 * is out of range, -3 if 2^31 - 1 rounds pass without emptying W. */
int oracle_jp(int32_t n, const int32_t *rowptr, const int32_t *colidx, uint64_t seed,
              int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
              int64_t *wsize, int64_t *arcs, int32_t stats_cap)
{
    *ncolors_out = 0;
    *rounds_out = 0;
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;
    int32_t *color = calloc((size_t)n, sizeof(int32_t));    /* 0 = still in W */
    uint64_t *r = calloc((size_t)n, sizeof(uint64_t));
    uint8_t *inS = calloc((size_t)n, 1);
    int32_t *W = malloc((size_t)n * sizeof(int32_t));
    if (!color || !r || !inS || !W) {
        free(color); free(r); free(inS); free(W);
        return -1;
    }
    int64_t wn = n;
    for (int32_t v = 0; v < n; ++v) W[v] = v;
    int32_t c = 0;
    while (wn > 0) {
        if (c == INT32_MAX) { free(color); free(r); free(inS); free(W); return -3; }
        ++c;
        int64_t a = 0;
        for (int64_t i = 0; i < wn; ++i) r[W[i]] = oracle_jp_priority(seed, c, W[i]);
        for (int64_t i = 0; i < wn; ++i) {
            int32_t v = W[i];
            int flag = 1;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (w != v && color[w] == 0 && r[v] <= r[w]) { flag = 0; break; }
            }
            inS[v] = (uint8_t)flag;
            a += rowptr[v + 1] - rowptr[v];
        }
        if (c - 1 < stats_cap) {
            if (wsize) wsize[c - 1] = wn;
            if (arcs) arcs[c - 1] = a;
        }
        int64_t nn = 0;
        for (int64_t i = 0; i < wn; ++i) {
            int32_t v = W[i];
            if (inS[v]) color[v] = c;
            else W[nn++] = v;
        }
        wn = nn;
    }
    for (int32_t v = 0; v < n; ++v) colors_out[v] = color[v] - 1;
    *ncolors_out = c;
    *rounds_out = c;
    free(color); free(r); free(inS); free(W);
    return 0;
}
