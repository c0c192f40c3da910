// Device-planned colouring: the whole run of Sec. 3.1 (Algorithm Data-GC) enqueued
// without any host read-back, so it can run behind the caller's stream or inside a
// captured hipGraph.
//
// The host-driven runs read the validation results back (bucket histogram, row order,
// arc count, split-row chunk count) to lay out the worklists and size the scratch.
// Here a one-thread plan kernel turns the same results into the argument blocks of the
// rounds (one per worklist parity) in device memory, checks that the graph fits the
// scratch the host provided, and the kernels after it read their arguments from there:
//   k_init -> k_validate_rows -> k_validate_arcs [-> k_validate_batch]
//   [-> k_check_symmetric] -> k_dev_plan -> k_dev_clear -> k_round1_dev
//   -> k_persistent_dev (every later round, device-wide barriers) -> k_dev_finish
// Every kernel after the plan returns at once when an error bit is set, and the finish
// kernel turns the error bits into a negative status in the caller's colour-count slot.
#pragma once

#include "sgr_kernels.h"

namespace csrcolor {

// What the host provides for a device-planned run (sizes in the units named).
struct DevCaps {
    long long f_words;         // words of the push-mode flag array F
    long long live_ints;       // ints of the live-list array (0: live lists off)
    long long split_ints;      // ints of the split-row scratch at `split`
    int* split;
    unsigned long long* lb1;   // ordered compaction: round-1 look-back status words, or null
    int lb1_ints;              // ints of lb1 to clear
    int want_live;             // live lists asked for (id rule, worklist rounds)
};

// The plan: the rounds' argument blocks and the extents the clearing kernel zeroes.
struct DevPlan {
    RoundArgs odd;             // rounds with odd 0-based index (the second round first): parity 1 -> 0
    RoundArgs even;            // parity 0 -> 1
    unsigned long long* lb1;
    long long f_words;         // F words to clear
    int hub_ints;              // split-row merge state to clear (bitmaps, done counters, lost flags)
    int dirty_words;           // dirty bytes to clear, as 4-byte words
    int lb1_ints;
    long long fq_words;        // small-colour flag slots to clear, as 4-byte words
};

// `t` holds everything the host knows (arrays, options; wl_in = wl[1], wl_out = wl[0]);
// the plan adds what only the device knows.  One thread.
__global__ void k_dev_plan(RoundArgs t, DevCaps c, DevPlan* p) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    Ctl* ctl = t.ctl;
    // the kernels after the plan find the control block (and its error bits) here, also
    // when the plan stops early; the rest of the block is only read once no error is set
    p->odd.ctl = ctl;
    p->even.ctl = ctl;
    if (ctl->err) return;
    const int n = t.n;
    const int nnz = ctl->nnz;
    RoundArgs a = t;
    a.nnz = nnz;
    a.sorted = ctl->desc_total == ctl->desc_bound;
    int hist[NB];
    for (int b = 0; b < NB; ++b) hist[b] = ctl->hist[b];
    a.seg[0] = 0;
    for (int b = 0; b < NB; ++b) a.seg[b + 1] = a.seg[b] + hist[b];
    const int nhub = hist[BSPLIT];
    const int nchunk = ctl->hchunks;
    const bool long_rows = hist[NTILE] + hist[NTILE + 1] + hist[BSPLIT] > 0;
    // live lists only change which arcs a test reads, never the colouring: a graph
    // whose arcs exceed their buffer runs without them
    const bool use_live = c.want_live && long_rows && (long long)max(nnz, 1) <= c.live_ints;
    long long fw = 0;
    if (a.pushff) {
        const long long flags = (long long)nnz + n;
        fw = a.pushff == 2 ? flags / 4 + 4 : flags / 32 + 2;
    }
    // (the same layout as the host-driven runs: chunk records first, 16-byte aligned)
    const long long recs = use_live ? 8LL * nchunk : 0;
    const long long split_ints = recs + 2LL * nhub + 2LL * nchunk + (long long)nhub * (HW + 4) +
                                 (use_live ? 2LL * nchunk : 0) + 2LL * nchunk;
    if (fw > c.f_words || split_ints > c.split_ints) {
        atomicOr(&ctl->err, ERR_NOMEM);
        return;
    }
    int4* crec0 = use_live ? reinterpret_cast<int4*>(c.split) : nullptr;
    int4* crec1 = use_live ? crec0 + nchunk : nullptr;
    int* cstart0 = c.split + recs;
    int* cstart1 = cstart0 + nhub;
    int* owner0 = cstart1 + nhub;
    int* owner1 = owner0 + nchunk;
    // per hub: HW bitmap words, then done counters, lost flags and 64-bit merge words
    int* hubflags = owner1 + nchunk;
    int* clen = use_live ? hubflags + (size_t)nhub * (HW + 4) : nullptr;
    int* cpos = use_live ? clen + nchunk : nullptr;
    int* settled = hubflags + (size_t)nhub * (HW + 4) + (use_live ? 2 * nchunk : 0);
    a.cstart[0] = cstart0;
    a.cstart[1] = cstart1;
    a.owner[0] = owner0;
    a.owner[1] = owner1;
    a.hubbm = reinterpret_cast<unsigned*>(hubflags);
    a.hubdone = hubflags + (size_t)nhub * HW;
    a.hublost = a.hubdone + nhub;
    a.hubst = reinterpret_cast<unsigned long long*>(a.hublost + nhub);
    a.crec[0] = crec0;
    a.crec[1] = crec1;
    a.settled = (a.pushff && nhub > 0) ? settled : nullptr;
    a.settled_k = settled + nchunk;
    a.live = use_live ? t.live : nullptr;
    a.llen = use_live ? t.llen : nullptr;
    a.clen = clen;
    a.lpos = use_live ? t.lpos : nullptr;
    a.cpos = cpos;
    if (!a.pushff) {
        a.F = nullptr;
        a.dirty = nullptr;
    }
    if (a.pushff != 2) a.Fq = nullptr;
    RoundArgs e = a;
    a.par_in = 1;
    a.par_out = 0;
    e.par_in = 0;
    e.par_out = 1;
    e.wl_in = t.wl_out;
    e.wl_out = const_cast<int*>(t.wl_in);
    p->odd = a;
    p->even = e;
    p->lb1 = c.lb1;
    p->lb1_ints = c.lb1 ? c.lb1_ints : 0;
    p->f_words = fw;
    p->hub_ints = nhub * (HW + 4);
    p->dirty_words = a.pushff ? n / 4 + 1 : 0;
    p->fq_words = a.Fq ? (long long)n * (KQ / 4) : 0;
}

// Zeroes what the plan asks for: the push flags, the split-row merge state, the dirty
// bytes, the round-1 look-back words and the small-colour flag slots (a kernel, not a
// memset, so it can be captured).
__global__ __launch_bounds__(WG) void k_dev_clear(const DevPlan* __restrict__ p) {
    const RoundArgs& a = p->odd;
    if (a.ctl->err) return;
    const long long fw = p->f_words;
    const long long hw = p->hub_ints;
    const long long dw = p->dirty_words;
    const long long lw = p->lb1_ints;
    const long long qw = p->fq_words;
    const long long tot = fw + hw + dw + lw + qw;
    const long long stride = (long long)gridDim.x * WG;
    int* F = reinterpret_cast<int*>(a.F);
    int* hub = reinterpret_cast<int*>(a.hubbm);
    int* dirty = reinterpret_cast<int*>(a.dirty);
    int* lb = reinterpret_cast<int*>(p->lb1);
    int* fq = reinterpret_cast<int*>(a.Fq);
    for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < tot; i += stride) {
        if (i < fw) F[i] = 0;
        else if (i < fw + hw) hub[i - fw] = 0;
        else if (i < fw + hw + dw) dirty[i - fw - hw] = 0;
        else if (i < fw + hw + dw + lw) lb[i - fw - hw - dw] = 0;
        else fq[i - fw - hw - dw - lw] = 0;
    }
}

// Round 1 (the all-colour-1 shortcut) with the planned arguments: it fills the parity-1
// worklists that the first persistent round reads.
__global__ __launch_bounds__(WG) void k_round1_dev(const DevPlan* __restrict__ p) {
    const RoundArgs& a = p->odd;
    if (a.ctl->err) return;
    round1_body(a.n, a.rowptr, a.colidx, a.X, a.out, const_cast<int*>(a.wl_in), a.ctl, a.sorted, a.twave,
                a.tsplit, a.seg, a.cstart[1], a.owner[1], a.F, a.nnz, a.rule, 0, a.hint, a.llen, a.clen, p->lb1,
                a.pushff == 2, a.dirty, nullptr, nullptr, nullptr, nullptr, a.Fq, a.crec[1], a.tiles);
}

// Every round after the first in one launch (persistent_rounds), arguments from the plan.
__global__ __launch_bounds__(WG) void k_persistent_dev(const DevPlan* __restrict__ p, int max_rounds,
                                                       long long limit) {
    if (p->odd.ctl->err) return;
    persistent_rounds(p->odd, p->even, 1, max_rounds, limit);
}

// Status of a finished device-planned run from the control block (0 = success).
__device__ __forceinline__ int dev_status(const Ctl* ctl) {
    const int e = ctl->err;
    if (e & (ERR_ROWPTR | ERR_COLIDX | ERR_MULTI | ERR_BATCH)) return -2;   // CSRCOLOR_EBADCSR
    if (e & ERR_ASYM) return -6;                                          // CSRCOLOR_ENOTSYM
    if (e & ERR_UNSORTED) return -1;                                      // CSRCOLOR_EINVAL
    if (e & ERR_NOMEM) return -3;                                         // CSRCOLOR_ENOMEM
    if (e & ERR_BARRIER) return -8;                                       // CSRCOLOR_ETIMEOUT
    if (e) return -4;                                                     // CSRCOLOR_EHIP
    if (!ctl->pdone) return -7;                                           // CSRCOLOR_ELIMIT
    return 0;
}

// Writes the colour counts: one graph (G == 0): ncolors[0] = the largest colour (vertex
// 0 always settles in round 1 with colour 1, which the device maximum does not see);
// G graphs of a block-diagonal union: ncolors[g] = 1 + the largest 0-based colour of
// graph g.  On an error every slot receives the negative status instead.
__global__ __launch_bounds__(WG) void k_dev_finish(const Ctl* __restrict__ ctl, int G,
                                                   const long long* __restrict__ voff,
                                                   const int* __restrict__ colors, int* ncolors) {
    __shared__ int red[WAVES];
    const int st = dev_status(ctl);
    if (G == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ncolors[0] = st ? st : max(ctl->maxcolor, 1);
        return;
    }
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        if (st) {
            if (threadIdx.x == 0) ncolors[g] = st;
            continue;
        }
        const long long v0 = voff[g], v1 = voff[g + 1];
        int m = -1;
        for (long long v = v0 + threadIdx.x; v < v1; v += WG) m = max(m, colors[v]);
        m = block_max(m, red);
        if (threadIdx.x == 0) ncolors[g] = m + 1;
    }
}

}  // namespace csrcolor
