/*
 * Serial CPU oracle for data-driven speculative-greedy (SGR) graph coloring.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (Chen et al., "Efficient and High-quality Sparse Graph
 * Coloring on GPUs", Sec. 3.1, Algorithm Data-GC built from the FirstFit and
 * ConflictResolve routines of Sec. 3, with colour clearing of Sec. 3.1):
 *
 *   S = snapshot colours, 0 = uncoloured (initial state of Sec. 2.1);
 *   W = V (the in-worklist starts as all vertices);
 *   while W is not empty:                         one round
 *     for v in W:  C[v] = smallest c > 0 not in { S[w] : w in adj(v), w != v }
 *     for v in W:  lose[v] = exists w in adj(v), w != v, w < v, C[w] == C[v]
 *     for v in W:  S[v] = lose[v] ? 0 : C[v]      (a loser's colour is cleared)
 *     W = { v in W : lose[v] }
 *
 * Readings taken where the paper leaves freedom (each listed in the design notes):
 *   - FirstFit reads only the previous round's snapshot S (Jacobi rounds), never a
 *     colour written earlier in the same round;
 *   - of two adjacent worklist vertices with equal tentative colour, the one with
 *     the HIGHER id is requeued (the printed ConflictResolve requeues the lower id;
 *     relabelling v -> n-1-v maps one rule onto the other);
 *   - the conflict test is pairwise on tentative colours, so a vertex is requeued by
 *     a lower neighbour even if that neighbour is itself requeued;
 *   - self-loops (w == v) are ignored; duplicate arcs are harmless.
 * Vertices outside W keep C[w] equal to their final colour, so a single C array
 * serves every round.
 *
 * Output colours are 0-based (S - 1); ncolors is the largest colour.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Per-round statistics (optional, any pointer may be NULL):
 *   wsize[r]  = |W_r|
 *   arcs_ff[r] = sum of row lengths over W_r (arcs scanned by FirstFit)
 *   arcs_cr[r] = arcs (v, w) with w < v examined by the conflict test when each row
 *                is scanned in storage order and the scan stops at the first
 *                conflict (and, for sorted rows, before the first w >= v).
 * Returns 0, or -1 if an allocation failed, -2 if a colidx entry is out of range. */
/* Conflict rules:
 *   rule 0 (id):     of two adjacent worklist vertices with equal tentative colour the
 *                    higher id is requeued;
 *   rule 1 (degree): the heuristic conflict resolve of Sec. 3.2: the vertex of larger
 *                    degree keeps its colour and the other is requeued; on equal degree
 *                    the smaller id keeps it (the higher id is requeued).
 * Degree = row length.  Under rule 1 every neighbour is examined (a higher-id
 * neighbour of larger degree can requeue v), so arcs_cr counts all examined arcs. */
static int beats(const int32_t *rowptr, int32_t w, int32_t v, int rule)
{
    if (rule == 0) return w < v;
    int64_t dw = rowptr[w + 1] - rowptr[w], dv = rowptr[v + 1] - rowptr[v];
    return dw > dv || (dw == dv && w < v);
}

int oracle_sgr_rule(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                    int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
                    int64_t *wsize, int64_t *arcs_ff, int64_t *arcs_cr, int32_t stats_cap, int32_t rule);

int oracle_sgr(int32_t n, const int32_t *rowptr, const int32_t *colidx,
               int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
               int64_t *wsize, int64_t *arcs_ff, int64_t *arcs_cr, int32_t stats_cap)
{
    return oracle_sgr_rule(n, rowptr, colidx, colors_out, ncolors_out, rounds_out,
                           wsize, arcs_ff, arcs_cr, stats_cap, 0);
}

/* As oracle_sgr_rule, stopping after max_rounds rounds when max_rounds > 0 (only to time
 * a bounded sample of a long colouring: colours of vertices still on the worklist then
 * read as -1, and *rounds_out counts the rounds run). */
int oracle_sgr_capped(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                      int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
                      int64_t *wsize, int64_t *arcs_ff, int64_t *arcs_cr, int32_t stats_cap, int32_t rule,
                      int32_t max_rounds);

int oracle_sgr_rule(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                    int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
                    int64_t *wsize, int64_t *arcs_ff, int64_t *arcs_cr, int32_t stats_cap, int32_t rule)
{
    return oracle_sgr_capped(n, rowptr, colidx, colors_out, ncolors_out, rounds_out, wsize, arcs_ff, arcs_cr,
                             stats_cap, rule, 0);
}

int oracle_sgr_capped(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                      int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
                      int64_t *wsize, int64_t *arcs_ff, int64_t *arcs_cr, int32_t stats_cap, int32_t rule,
                      int32_t max_rounds)
{
    *ncolors_out = 0;
    *rounds_out = 0;
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;

    int32_t *S = calloc((size_t)n, sizeof(int32_t));
    int32_t *C = calloc((size_t)n, sizeof(int32_t));
    int32_t *W = malloc((size_t)n * sizeof(int32_t));
    int32_t *Wn = malloc((size_t)n * sizeof(int32_t));
    uint8_t *lose = calloc((size_t)n, 1);
    /* colour-indexed stamp array: stamp[c] == v+1 means colour c is forbidden to v */
    int64_t *stamp = calloc((size_t)n + 2, sizeof(int64_t));
    if (!S || !C || !W || !Wn || !lose || !stamp) {
        free(S); free(C); free(W); free(Wn); free(lose); free(stamp);
        return -1;
    }
    int sorted = 1;
    for (int32_t v = 0; v < n && sorted; ++v)
        for (int64_t e = rowptr[v] + 1; e < rowptr[v + 1]; ++e)
            if (colidx[e] < colidx[e - 1]) { sorted = 0; break; }

    int64_t wn = n;
    for (int32_t v = 0; v < n; ++v) W[v] = v;
    int32_t r = 0;
    while (wn > 0 && (max_rounds <= 0 || r < max_rounds)) {
        int64_t aff = 0, acr = 0;
        /* FirstFit on every worklist vertex, against the snapshot S */
        for (int64_t i = 0; i < wn; ++i) {
            int32_t v = W[i];
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (w != v) stamp[S[w]] = (int64_t)v + 1;
            }
            aff += rowptr[v + 1] - rowptr[v];
            int32_t c = 1;
            while (stamp[c] == (int64_t)v + 1) ++c;
            C[v] = c;
        }
        /* conflict test: a neighbour that beats v (rule 0: lower id) holding the same
           tentative colour */
        for (int64_t i = 0; i < wn; ++i) {
            int32_t v = W[i];
            lose[v] = 0;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (w == v) continue;
                if (rule == 0 && w > v) {
                    if (sorted) break;
                    continue;
                }
                ++acr;
                if (C[w] == C[v] && beats(rowptr, w, v, rule)) { lose[v] = 1; break; }
            }
        }
        /* winners keep their colour, losers are cleared and requeued */
        int64_t nn = 0;
        for (int64_t i = 0; i < wn; ++i) {
            int32_t v = W[i];
            if (lose[v]) { S[v] = 0; Wn[nn++] = v; }
            else S[v] = C[v];
        }
        if (r < stats_cap) {
            if (wsize) wsize[r] = wn;
            if (arcs_ff) arcs_ff[r] = aff;
            if (arcs_cr) arcs_cr[r] = acr;
        }
        ++r;
        int32_t *t = W; W = Wn; Wn = t;
        wn = nn;
    }
    int32_t mx = 0;
    for (int32_t v = 0; v < n; ++v) {
        colors_out[v] = S[v] - 1;
        if (S[v] > mx) mx = S[v];
    }
    *ncolors_out = mx;
    *rounds_out = r;
    free(S); free(C); free(W); free(Wn); free(lose); free(stamp);
    return 0;
}

/* Topology-driven variant (Sec. 3.1, Algorithm Topo-GC): every round visits every
 * vertex; an uncoloured one (colour 0) runs FirstFit against the previous round's
 * colours, and every vertex not yet marked coloured runs the conflict test and is
 * marked coloured when it has no conflict.  The loop ends after a round in which no
 * vertex was uncoloured.  Same readings as oracle_sgr_rule (snapshot FirstFit,
 * pairwise test, loser cleared, rule 0/1 requeue direction).  Statistics per round:
 * wsize[r] = vertices that ran FirstFit, visits[r] = vertices visited (always n).
 * The worklist of the data-driven algorithm is exactly the set of uncoloured
 * vertices, so the colouring must equal oracle_sgr_rule's. */
int oracle_sgr_topo(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                    int32_t *colors_out, int32_t *ncolors_out, int32_t *rounds_out,
                    int64_t *wsize, int64_t *visits, int32_t stats_cap, int32_t rule)
{
    *ncolors_out = 0;
    *rounds_out = 0;
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;
    int32_t *color = calloc((size_t)n, sizeof(int32_t));   /* 0 = uncoloured */
    int32_t *tent = calloc((size_t)n, sizeof(int32_t));    /* this round's FirstFit result */
    uint8_t *colored = calloc((size_t)n, 1);
    uint8_t *lose = calloc((size_t)n, 1);
    int64_t *stamp = calloc((size_t)n + 2, sizeof(int64_t));
    if (!color || !tent || !colored || !lose || !stamp) {
        free(color); free(tent); free(colored); free(lose); free(stamp);
        return -1;
    }
    int32_t r = 0;
    for (;;) {
        int64_t ran = 0;
        /* FirstFit over V for the uncoloured vertices, reading last round's colours */
        for (int32_t v = 0; v < n; ++v) {
            if (color[v] != 0) { tent[v] = color[v]; continue; }
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (w != v) stamp[color[w]] = (int64_t)v + 1;
            }
            int32_t c = 1;
            while (stamp[c] == (int64_t)v + 1) ++c;
            tent[v] = c;
            ++ran;
        }
        if (ran == 0) break;
        /* conflict test over V for the vertices not yet marked coloured */
        for (int32_t v = 0; v < n; ++v) {
            lose[v] = 0;
            if (colored[v]) continue;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (w != v && tent[w] == tent[v] && beats(rowptr, w, v, rule)) {
                    lose[v] = 1;
                    break;
                }
            }
        }
        for (int32_t v = 0; v < n; ++v) {
            if (colored[v]) continue;
            if (lose[v]) color[v] = 0;
            else { color[v] = tent[v]; colored[v] = 1; }
        }
        if (r < stats_cap) {
            if (wsize) wsize[r] = ran;
            if (visits) visits[r] = n;
        }
        ++r;
    }
    int32_t mx = 0;
    for (int32_t v = 0; v < n; ++v) {
        colors_out[v] = color[v] - 1;
        if (color[v] > mx) mx = color[v];
    }
    *ncolors_out = mx;
    *rounds_out = r;
    free(color); free(tent); free(colored); free(lose); free(stamp);
    return 0;
}

/* Sequential greedy colouring in natural vertex order (Sec. 2.1, Algorithm 1):
 * vertex v takes the smallest positive colour not held by an already-coloured
 * neighbour.  Output colours are 0-based.  Returns -2 if a colidx entry is out of
 * range. */
int oracle_serial_ff(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                     int32_t *colors_out, int32_t *ncolors_out)
{
    *ncolors_out = 0;
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;
    int32_t *col = calloc((size_t)n, sizeof(int32_t));
    int64_t *stamp = calloc((size_t)n + 2, sizeof(int64_t));
    if (!col || !stamp) { free(col); free(stamp); return -1; }
    int32_t mx = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            int32_t w = colidx[e];
            if (w != v) stamp[col[w]] = (int64_t)v + 1;
        }
        int32_t c = 1;
        while (stamp[c] == (int64_t)v + 1) ++c;
        col[v] = c;
        if (c > mx) mx = c;
    }
    for (int32_t v = 0; v < n; ++v) colors_out[v] = col[v] - 1;
    *ncolors_out = mx;
    free(col); free(stamp);
    return 0;
}

/* Number of arcs (v, w), v != w, whose endpoints share a colour (0 = proper); -2 if a
 * colidx entry is out of range. */
int64_t oracle_count_conflicts(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                               const int32_t *colors)
{
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;
    int64_t bad = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            int32_t w = colidx[e];
            if (w != v && colors[w] == colors[v]) ++bad;
        }
    return bad;
}

/* Number of vertices whose colour is not the smallest colour absent from its
 * neighbourhood (0-based colours; 0 = the colouring is a Grundy colouring); -2 if a
 * colidx entry is out of range. */
int64_t oracle_count_non_grundy(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                                const int32_t *colors)
{
    if (n <= 0) return 0;
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return -2;
    int64_t *stamp = calloc((size_t)n + 2, sizeof(int64_t));
    if (!stamp) return -1;
    int64_t bad = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            int32_t w = colidx[e];
            if (w != v && colors[w] >= 0 && colors[w] <= n) stamp[colors[w]] = (int64_t)v + 1;
        }
        int32_t c = 0;
        while (stamp[c] == (int64_t)v + 1) ++c;
        if (c != colors[v]) ++bad;
    }
    free(stamp);
    return bad;
}
