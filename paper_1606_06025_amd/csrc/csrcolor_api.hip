// Host driver and C-ABI of the speculative-greedy colouring library.
//
// One colouring (Sec. 3.1, Algorithm Data-GC):
//   k_init -> k_validate_rows -> k_validate_arcs -> [read back: errors, degree
//   histogram, max degree, row order] (-> k_check_symmetric -> [read back])
//   -> k_round1 -> { k_assign ; k_detect } per round, the worklist length read back
//   every few rounds -> [read back: colour count].
// Worklists are double-buffered by round parity (Sec. 3.1, swap of W_in / W_out);
// each degree bucket owns a fixed segment of both worklist arrays whose size is the
// number of vertices of that bucket, so no push can overflow.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/csrcolor.h"
#include "sgr_kernels.h"
#include "sgr_plan.h"
#include "sgr_topo.h"

namespace csrcolor {
namespace {

struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    size_t cap_n = 0;            // vertices the arrays below can hold
    int* X = nullptr;            // colour state
    int* wl[2] = {nullptr, nullptr};
    int* hint = nullptr;         // conflict hints: a neighbour that beat the vertex
    int* llen = nullptr;         // live-list lengths (or a split row's chunk-slot base)
    int* lpos = nullptr;         // live lists: resume positions in the rows
    unsigned char* Fq = nullptr; // push FirstFit, byte flags: KQ flag bytes per vertex (colours 1..KQ)
    unsigned char* dirty = nullptr;   // push FirstFit: flags changed since the last FirstFit
    unsigned char* rflag = nullptr;   // wake flags: recolour this round (padded to whole scans)
    unsigned char* aflag = nullptr;   // wake flags: test this round (padded likewise)
    int* srnd = nullptr;              // wake flags: settling round per vertex
    unsigned long long* Fs = nullptr; // wake flags: forbidden-colour masks of the short rows
    unsigned long long* ubytes = nullptr;   // wake flags: bytes moved by the two kernels (on request)
    int* live = nullptr;         // live lists, same offsets as colidx
    size_t live_cap = 0;         // ints
    unsigned long long* lb = nullptr;   // look-back status words of ordered compaction
    size_t lb_cap = 0;
    Ctl* ctl = nullptr;          // device control block
    Ctl* ctl_h = nullptr;        // pinned host mirror
    Ctl* ctl_h2 = nullptr;       // second pinned mirror: read-backs that overlap the next rounds
    hipEvent_t pev[2] = {nullptr, nullptr};
    int st_cap = 0;
    long long* st_wsize = nullptr;
    long long* st_arcs = nullptr;
    // split-row bucket scratch: cstart[2] and hub flags sized by hub count, owner[2] by chunk count
    int* split = nullptr;
    size_t split_cap = 0;        // ints
    unsigned* F = nullptr;       // push-mode forbidden-colour bitmaps
    size_t F_cap = 0;            // words
    // multi-graph calls: union CSR, its colours, vertex offsets and the graph table
    int* u_rowptr = nullptr;
    int* u_colidx = nullptr;
    int* u_colors = nullptr;
    long long* u_voff = nullptr;
    MultiDesc* u_desc = nullptr;
    MultiDesc* u_desc_h = nullptr;   // pinned staging for the table
    long long* u_voff_h = nullptr;   // pinned staging for the offsets
    size_t u_n_cap = 0, u_e_cap = 0, u_g_cap = 0;
    std::vector<hipEvent_t> evs; // event pool for per-kernel timing
    // graph mode: private capture stream, the instantiated two-round graph and the
    // arguments it was captured with
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    hipGraphExec_t gexec = nullptr;
    RoundArgs gargs;
    int gbudget = 0;
    // device-planned runs: the plan block, the largest arc count the arc-sized buffers
    // (flags, live lists, split-row scratch) were sized for, and a pinned word for the
    // sizing read of rowptr[n]
    DevPlan* plan = nullptr;
    long long arc_cap = 0;
    int* sz_h = nullptr;
    std::mutex mu;
};

// Times kernel launches on the workspace stream when enabled.  A single kernel goes
// through hipExtLaunchKernelGGL, whose start and stop events take the timestamps of
// the dispatch itself (the kernel's own execution time, as a kernel trace reports
// it); a group of launches is bracketed by events recorded on the stream.
struct KTimer {
    Workspace* w;
    bool on;
    size_t next = 0;
    std::vector<std::pair<size_t, size_t>> spans[3];   // 0 setup, 1 assign, 2 detect
    KTimer(Workspace* ws, bool enable) : w(ws), on(enable) {}
    size_t event() {
        if (next == w->evs.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { on = false; return 0; }
            w->evs.push_back(e);
        }
        return next++;
    }
    size_t mark() {
        const size_t i = event();
        if (on) (void)hipEventRecord(w->evs[i], w->stream);
        return i;
    }
    template <class F>
    void run(int kind, F&& launch) {
        if (!on) { launch(); return; }
        const size_t a = mark();
        launch();
        const size_t b = mark();
        if (on) spans[kind].push_back({a, b});
    }
    template <class K, class... A>
    void kern(int kind, K kernel, int grid, int block, A... args) {
        if (on) {
            const size_t a = event();
            const size_t b = event();
            if (on) {
                hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, w->stream, w->evs[a], w->evs[b], 0,
                                      args...);
                spans[kind].push_back({a, b});
                return;
            }
        }
        kernel<<<grid, block, 0, w->stream>>>(args...);
    }
    double total_ms(int kind, int* count) const {
        double t = 0;
        for (auto& p : spans[kind]) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, w->evs[p.first], w->evs[p.second]) == hipSuccess) t += ms;
        }
        if (count) *count = (int)spans[kind].size();
        return t;
    }
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
int g_num_cus[64] = {0};

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return CSRCOLOR_EHIP;     \
    } while (0)

int num_cus(int dev) {
    if (dev < 0 || dev >= 64) return 256;
    if (g_num_cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        g_num_cus[dev] = c;
    }
    return g_num_cus[dev];
}

// Workgroups of a conflict-test launch: the budget, at most DETECT_PER_CU per CU.
int detect_grid(int dev, int budget) { return std::max(1, std::min(budget, num_cus(dev) * DETECT_PER_CU)); }

Workspace* get_ws(int dev, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = stream;
    g_ws[key] = w;
    return w;
}

void free_union(Workspace* w) {
    if (w->u_rowptr) (void)hipFree(w->u_rowptr);
    if (w->u_colidx) (void)hipFree(w->u_colidx);
    if (w->u_colors) (void)hipFree(w->u_colors);
    if (w->u_voff) (void)hipFree(w->u_voff);
    if (w->u_desc) (void)hipFree(w->u_desc);
    if (w->u_desc_h) (void)hipHostFree(w->u_desc_h);
    if (w->u_voff_h) (void)hipHostFree(w->u_voff_h);
    w->u_rowptr = w->u_colidx = w->u_colors = nullptr;
    w->u_voff = nullptr;
    w->u_desc = w->u_desc_h = nullptr;
    w->u_voff_h = nullptr;
    w->u_n_cap = w->u_e_cap = w->u_g_cap = 0;
}

int ensure_union(Workspace* w, size_t N, size_t E, size_t G) {
    if (N <= w->u_n_cap && E <= w->u_e_cap && G <= w->u_g_cap) return CSRCOLOR_OK;
    (void)hipStreamSynchronize(w->stream);
    const size_t n2 = std::max(N, w->u_n_cap), e2 = std::max(E, w->u_e_cap), g2 = std::max(G, w->u_g_cap);
    free_union(w);
    if (hipMalloc(&w->u_rowptr, (n2 + 1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&w->u_colidx, std::max(e2, (size_t)1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&w->u_colors, std::max(n2, (size_t)1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&w->u_voff, (g2 + 1) * sizeof(long long)) != hipSuccess ||
        hipMalloc(&w->u_desc, g2 * sizeof(MultiDesc)) != hipSuccess ||
        hipHostMalloc(&w->u_desc_h, g2 * sizeof(MultiDesc), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&w->u_voff_h, (g2 + 1) * sizeof(long long), hipHostMallocDefault) != hipSuccess) {
        free_union(w);
        return CSRCOLOR_ENOMEM;
    }
    w->u_n_cap = n2;
    w->u_e_cap = e2;
    w->u_g_cap = g2;
    return CSRCOLOR_OK;
}

// Frees only the per-vertex arrays (colour state and worklists).  Every other
// buffer of the workspace has its own ensure_* / free pair, so growing one never
// invalidates another that the caller has already filled.
void free_vertex_arrays(Workspace* w) {
    if (w->X) (void)hipFree(w->X);
    if (w->wl[0]) (void)hipFree(w->wl[0]);
    if (w->wl[1]) (void)hipFree(w->wl[1]);
    if (w->hint) (void)hipFree(w->hint);
    if (w->llen) (void)hipFree(w->llen);
    if (w->lpos) (void)hipFree(w->lpos);
    if (w->Fq) (void)hipFree(w->Fq);
    w->Fq = nullptr;
    if (w->dirty) (void)hipFree(w->dirty);
    if (w->rflag) (void)hipFree(w->rflag);
    if (w->aflag) (void)hipFree(w->aflag);
    if (w->srnd) (void)hipFree(w->srnd);
    if (w->Fs) (void)hipFree(w->Fs);
    w->rflag = w->aflag = nullptr;
    w->srnd = nullptr;
    w->Fs = nullptr;
    w->X = w->wl[0] = w->wl[1] = w->hint = w->llen = w->lpos = nullptr;
    w->dirty = nullptr;
    w->cap_n = 0;
}

// Frees every device array of the workspace (release_workspace).
void free_ws_arrays(Workspace* w) {
    free_union(w);
    w->arc_cap = 0;
    if (w->F) (void)hipFree(w->F);
    w->F = nullptr;
    w->F_cap = 0;
    if (w->split) (void)hipFree(w->split);
    w->split = nullptr;
    w->split_cap = 0;
    if (w->live) (void)hipFree(w->live);
    w->live = nullptr;
    w->live_cap = 0;
    if (w->lb) (void)hipFree(w->lb);
    w->lb = nullptr;
    w->lb_cap = 0;
    free_vertex_arrays(w);
}

// Bytes of a wake-flag array for n vertices: whole scans of VPW vertices, zero padded.
size_t flag_bytes(size_t n) { return (n + VPW - 1) / VPW * VPW + VPW; }

// Device bytes of the per-vertex arrays for `cap` vertices (ensure_capacity).
size_t vertex_bytes(size_t cap) {
    return cap * (7 * sizeof(int) + sizeof(unsigned long long) + KQ + 1) + 16 + 2 * flag_bytes(cap);
}

// Device bytes a workspace holds now, from the capacities it was allocated with.
size_t ws_bytes_now(const Workspace* w) {
    size_t b = 0;
    if (w->ctl) b += sizeof(Ctl) + 2 * sizeof(unsigned long long);
    if (w->cap_n) b += vertex_bytes(w->cap_n);
    b += w->F_cap * sizeof(unsigned) + w->split_cap * sizeof(int) + w->live_cap * sizeof(int) +
         w->lb_cap * sizeof(unsigned long long) + (size_t)w->st_cap * 2 * sizeof(long long);
    if (w->plan) b += sizeof(DevPlan);
    if (w->u_rowptr)
        b += (w->u_n_cap + 1) * sizeof(int) + std::max(w->u_e_cap, (size_t)1) * sizeof(int) +
             std::max(w->u_n_cap, (size_t)1) * sizeof(int) + (w->u_g_cap + 1) * sizeof(long long) +
             w->u_g_cap * sizeof(MultiDesc);
    return b;
}

// Upper bound of the device bytes one workspace needs to colour a graph of n vertices
// and nnz arcs (G > 0: a union of G graphs given to csrcolor_color_multi, whose copy
// the workspace also holds), for every option except statistics and ordered
// compaction: the allocations of ensure_capacity, ensure_F, ensure_split, ensure_live
// and ensure_union at the sizes either drive path asks for.
size_t ws_bound(long long G, long long n, long long nnz) {
    const size_t cap = std::max<size_t>((size_t)n, 1024);
    const size_t e = (size_t)std::max<long long>(nnz, 0);
    size_t b = sizeof(Ctl) + 2 * sizeof(unsigned long long) + sizeof(DevPlan) + vertex_bytes(cap);
    b += std::max<size_t>((cap + e) / 4 + 4, 4096) * sizeof(unsigned);      // push flags
    b += std::max<size_t>(e / 16 + 64, 4096) * sizeof(int);                 // split-row scratch
    b += std::max<size_t>(e, 4096) * sizeof(int);                           // live lists
    if (G > 0)
        b += ((size_t)n + 1) * sizeof(int) + std::max<size_t>(e, 1) * sizeof(int) +
             std::max<size_t>((size_t)n, 1) * sizeof(int) + ((size_t)G + 1) * sizeof(long long) +
             (size_t)G * sizeof(MultiDesc);
    return b;
}

int ensure_capacity(Workspace* w, size_t n, int st_cap) {
    if (!w->ctl) {
        HIP_TRY(hipMalloc(&w->ctl, sizeof(Ctl)));
        HIP_TRY(hipMalloc(&w->ubytes, 2 * sizeof(unsigned long long)));
        if (hipHostMalloc(&w->ctl_h, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return CSRCOLOR_ENOMEM;
    }
    if (n > w->cap_n) {
        (void)hipStreamSynchronize(w->stream);
        free_vertex_arrays(w);
        size_t want = std::max(n, (size_t)1024);
        if (hipMalloc(&w->X, want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->wl[0], want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->wl[1], want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->hint, want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->llen, want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->lpos, want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->Fq, want * KQ) != hipSuccess ||
            hipMalloc(&w->rflag, flag_bytes(want)) != hipSuccess ||
            hipMalloc(&w->aflag, flag_bytes(want)) != hipSuccess ||
            hipMalloc(&w->srnd, want * sizeof(int)) != hipSuccess ||
            hipMalloc(&w->Fs, want * sizeof(unsigned long long)) != hipSuccess ||
            hipMalloc(&w->dirty, want + 16) != hipSuccess) {
            free_vertex_arrays(w);
            return CSRCOLOR_ENOMEM;
        }
        w->cap_n = want;
    }
    if (st_cap > w->st_cap) {
        (void)hipStreamSynchronize(w->stream);
        if (w->st_wsize) (void)hipFree(w->st_wsize);
        if (w->st_arcs) (void)hipFree(w->st_arcs);
        w->st_wsize = w->st_arcs = nullptr;
        w->st_cap = 0;
        if (hipMalloc(&w->st_wsize, st_cap * sizeof(long long)) != hipSuccess ||
            hipMalloc(&w->st_arcs, st_cap * sizeof(long long)) != hipSuccess)
            return CSRCOLOR_ENOMEM;
        w->st_cap = st_cap;
    }
    return CSRCOLOR_OK;
}

int ensure_split(Workspace* w, size_t ints) {
    if (ints <= w->split_cap) return CSRCOLOR_OK;
    (void)hipStreamSynchronize(w->stream);
    if (w->split) (void)hipFree(w->split);
    w->split = nullptr;
    w->split_cap = 0;
    const size_t want = std::max(ints, (size_t)4096);
    if (hipMalloc(&w->split, want * sizeof(int)) != hipSuccess) return CSRCOLOR_ENOMEM;
    w->split_cap = want;
    return CSRCOLOR_OK;
}

int ensure_F(Workspace* w, size_t words) {
    if (words <= w->F_cap) return CSRCOLOR_OK;
    (void)hipStreamSynchronize(w->stream);
    if (w->F) (void)hipFree(w->F);
    w->F = nullptr;
    w->F_cap = 0;
    const size_t want = std::max(words, (size_t)4096);
    if (hipMalloc(&w->F, want * sizeof(unsigned)) != hipSuccess) return CSRCOLOR_ENOMEM;
    w->F_cap = want;
    return CSRCOLOR_OK;
}

int ensure_live(Workspace* w, size_t ints) {
    if (ints <= w->live_cap) return CSRCOLOR_OK;
    (void)hipStreamSynchronize(w->stream);
    if (w->live) (void)hipFree(w->live);
    w->live = nullptr;
    w->live_cap = 0;
    const size_t want = std::max(ints, (size_t)4096);
    if (hipMalloc(&w->live, want * sizeof(int)) != hipSuccess) return CSRCOLOR_ENOMEM;
    w->live_cap = want;
    return CSRCOLOR_OK;
}

int ensure_lb(Workspace* w, size_t words) {
    if (words <= w->lb_cap) return CSRCOLOR_OK;
    (void)hipStreamSynchronize(w->stream);
    if (w->lb) (void)hipFree(w->lb);
    w->lb = nullptr;
    w->lb_cap = 0;
    const size_t want = std::max(words, (size_t)16384);
    if (hipMalloc(&w->lb, want * sizeof(unsigned long long)) != hipSuccess) return CSRCOLOR_ENOMEM;
    w->lb_cap = want;
    return CSRCOLOR_OK;
}

int read_ctl(Workspace* w) {
    HIP_TRY(hipMemcpyAsync(w->ctl_h, w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return CSRCOLOR_OK;
}

struct Options {
    int mode = CSRCOLOR_MODE_LOOP;
    int validate = 0;
    int twave = 1024;
    int tiles = TILES_DEFAULT;
    int blocks_per_cu = 6;
    int sync_every = 8;
    int tsplit = 2048;
    int lane_assign = 0;      // tile buckets run with 2/4/8/16 lanes per vertex
    int lane_detect = 0;      // conflict test of the tile buckets: 0 lane-streamed (id rule); with bit 4
                              // set, L lanes per untested vertex, or for the buckets of bits 0-3 one
                              // lane per vertex without refill
    int pushff = 2;           // FirstFit: 0 rescan, 1 push with bit flags, 2 push with byte flags
    int hints = 1;            // conflict hints (id rule)
    int live = 1;             // live lists for degree > 61 (id rule)
    int ordered = 0;          // order-preserving worklist compaction (measured slower on the stencil)
    int wake = 0;             // wake flags: 0 auto (on when rows longer than 61 arcs hold under a
                              // tenth of the arcs), 1 on, -1 off (id rule, push FirstFit, hints,
                              // LOOP mode, unordered compaction)
    int rule = 0;             // conflict rule (csrcolor_rule)
    int algo = CSRCOLOR_ALGO_SGR;
    unsigned long long seed = 0;
};

// Range checks shared by the entry points; `single` is false for the batched and
// multi-graph calls, which do not take JP (its priorities depend on global ids).
bool opts_valid(const csrcolor_opts* o, bool single) {
    if (!o) return true;
    if (o->mode < 0 || o->mode > CSRCOLOR_MODE_GRAPH || o->validate < 0 || o->firstfit < 0 || o->firstfit > 3 ||
        o->rule < 0 || o->rule > 1 || o->algorithm < 0 || o->algorithm > CSRCOLOR_ALGO_JP || o->hints < -1 ||
        o->hints > 1 || o->live_lists < -1 || o->live_lists > 1 ||
        o->ordered < -1 || o->ordered > 1 || o->wake < -1 || o->wake > 1)
        return false;
    if (o->algorithm != CSRCOLOR_ALGO_SGR && (o->mode == CSRCOLOR_MODE_PERSISTENT || o->mode == CSRCOLOR_MODE_GRAPH))
        return false;
    if (o->tile_limits) {
        const int t0 = o->tile_limits & 0xff, t1 = (o->tile_limits >> 8) & 0xff, t2 = (o->tile_limits >> 16) & 0xff;
        if ((o->tile_limits >> 24) != 0 || t0 > 5 || t1 > 13 || t2 > 29 || t0 > t1 || t1 > t2) return false;
    }
    if (!single && o->algorithm == CSRCOLOR_ALGO_JP) return false;
    return true;
}

Options parse_opts(const csrcolor_opts* o) {
    Options r;
    if (!o) return r;
    if (o->mode) r.mode = o->mode;
    r.validate = o->validate;
    if (o->t_wave > 0) r.twave = std::min(std::max(o->t_wave, TWAVE_MIN), TWAVE_MAX);
    if (o->blocks_per_cu > 0) r.blocks_per_cu = std::min(o->blocks_per_cu, 32);
    if (o->sync_every > 0) r.sync_every = std::min(o->sync_every, 256);
    if (o->t_split > 0) r.tsplit = std::max(o->t_split, TSPLIT_MIN);
    if (o->tile_limits) r.tiles = o->tile_limits;
    r.tsplit = std::max(r.tsplit, r.twave);
    if (o->lane_assign) r.lane_assign = o->lane_assign < 0 ? 0 : (o->lane_assign & 0xF);
    if (o->lane_detect) r.lane_detect = o->lane_detect < 0 ? 0x10 : (0x10 | (o->lane_detect & 0xF));
    if (o->firstfit) r.pushff = o->firstfit - 1;
    if (o->hints) r.hints = o->hints > 0;
    if (o->live_lists) r.live = o->live_lists > 0;
    if (o->ordered) r.ordered = o->ordered > 0;
    r.wake = o->wake;
    r.rule = o->rule;
    r.algo = o->algorithm;
    r.seed = ((unsigned long long)o->seed_hi << 32) | o->seed_lo;
    if (r.algo != CSRCOLOR_ALGO_SGR) r.mode = CSRCOLOR_MODE_LOOP;
    if (r.algo == CSRCOLOR_ALGO_JP) {
        r.rule = RULE_JP;
        r.pushff = 0;
    }
    return r;
}

// Workgroups per bucket for the next rounds of the host loop, from upper bounds `ub`
// on the queue sizes (sizes only shrink from round to round; ub[BSPLIT] counts
// chunks).  Each bucket gets a share of the budget proportional to its estimated arc
// work (plan_cost), never more workgroups than it has units for.
void make_plan(const int ub[NB], int budget, int boff[NB + 1]) {
    double tot = 0;
    for (int b = 0; b < NB; ++b) tot += (double)ub[b] * plan_cost(b, 1);
    boff[0] = 0;
    for (int b = 0; b < NB; ++b) {
        int nb = 0;
        if (ub[b] > 0) {
            const double share = tot > 0 ? ub[b] * plan_cost(b, 1) / tot : 1.0;
            nb = std::max(1, (int)(share * budget + 0.5));
            const int useful = (ub[b] + plan_units_per_block(b) - 1) / plan_units_per_block(b);
            nb = std::min(nb, std::max(useful, 1));
            // buckets that flush per workgroup: at most SUB entries per block, so the
            // conflict test can keep the worklist order
            if (b <= NTILE) nb = std::max(nb, (ub[b] + SUB - 1) / SUB);
        }
        boff[b + 1] = boff[b] + nb;
    }
}

struct Job {
    int n;
    const int* rowptr;
    const int* colidx;
    int* colors_out;
    Options opt;
    csrcolor_stats* stats;
    // results
    int ncolors = 0;
    int rounds = 0;
    int sorted = 1;
    bool wake = false;       // the rounds ran with wake flags (statistics from settling rounds)
    int maxdeg = 0;
    long long nnz = 0;
    long long expect_nnz = -1;   // the caller's arc count, checked against rowptr[n] (-1: none given)
};

// Host loop: k_assign + k_detect per round with a host-computed partition; the queue
// sizes are read back every few rounds (2, 4, 8, ... up to sync_every).  Rounds
// launched past the end find empty queues and do nothing.
int drive_loop(Workspace* w, Job& J, RoundArgs& a, int ub[NB], int budget, KTimer& T) {
    int par = 1;             // parity of the worklist holding W of the next round
    const bool jp = a.rule == RULE_JP;
    long long launched = jp ? 0 : 1;   // rounds enqueued so far (SGR round 1 is k_round1)
    int k = 2;
    a.dev_plan = 0;
    for (;;) {
        long long tot = 0;
        for (int b = 0; b < NB; ++b) tot += ub[b];
        if (tot == 0) break;
        make_plan(ub, budget, a.boff);
        const int grid = a.boff[NB];
        a.lbs_n = budget;      // the conflict test runs on the whole budget (device partition)
        // push-mode FirstFit does little per entry (mostly a dirty-byte check), so it runs
        // on a smaller grid: fewer blocks to dispatch, more entries in flight per wavefront
        int aboff[NB + 1];
        for (int b = 0; b <= NB; ++b) aboff[b] = a.boff[b];
        if (a.pushff) make_plan(ub, std::max(budget / 3, 1), aboff);
        const int agrid = aboff[NB];
        for (int i = 0; i < k; ++i) {
            a.par_in = par;
            a.par_out = par ^ 1;
            a.wl_in = w->wl[par];
            a.wl_out = w->wl[par ^ 1];
            if (jp) {
                a.jpc = (int)launched + 1;    // colour of this JP round
                T.kern(1, k_jp_prep, 1, 256, a.ctl, a.par_out, a.lbs, grid);
            } else {
                RoundArgs aa = a;
                for (int b = 0; b <= NB; ++b) aa.boff[b] = aboff[b];
                T.kern(1, k_assign, agrid, WG, aa);
            }
            {
                // the conflict test partitions its grid by the exact queue sizes on the
                // device (the host only has upper bounds from earlier read-backs)
                RoundArgs ad = a;
                ad.dev_plan = 1;
                ad.lbs_n = budget;
                T.kern(2, k_detect<false>, detect_grid(w->device, budget), WG, ad);
            }
            if (a.pushff && ub[BSPLIT] > 0) {
                const int pg = std::min(ub[BSPLIT], budget);
                T.kern(2, k_push<false>, pg, WG, a);
            }
            par ^= 1;
            ++launched;
        }
        HIP_TRY(hipGetLastError());
        int rc = read_ctl(w);
        if (rc) return rc;
        if (w->ctl_h->err) return CSRCOLOR_EHIP;
        long long left = 0;
        for (int b = 0; b < NB; ++b) left += (ub[b] = w->ctl_h->cnt[par][b]);
        ub[BSPLIT] = w->ctl_h->ccnt[par];
        if (left > 0 && launched > (long long)J.n + 2) return CSRCOLOR_ELIMIT;   // rounds <= n
        k = std::min(k * 2, J.opt.sync_every);
    }
    return CSRCOLOR_OK;
}

// Host loop with wake flags: per round the recolouring FirstFit and the conflict test,
// both scanning the flag bytes of every vertex (plus the worklists of the long rows,
// device-side partition) and, when split rows exist, their push phase.  The conflict
// test stores the round number when it tests a vertex; a round that tests none means
// every vertex is settled (the lowest uncoloured vertex is always tested).  That is
// read back after every batch of rounds, one batch behind; rounds launched past the end
// do nothing.
// Launch shape of the flag scans: about 4096 wavefronts per scan (fewer leave the chip
// idle, more pay their fixed costs (launch, flag load, compaction) on mostly empty
// ranges; measured on the stencil: 2.1 M vertices best at 512 per wavefront, 0.9 M at
// 256).
void wake_shape(RoundArgs& a, int n, int budget) {
    a.vpw = 64;
    while (a.vpw < VPW && (long long)a.vpw * 4096 < n) a.vpw *= 2;
    const long long scans = ((long long)n + (long long)a.vpw * WAVES - 1) / ((long long)a.vpw * WAVES);
    a.gdense = (int)std::max<long long>(1, std::min<long long>(scans, 4LL * budget));
}

int drive_wake(Workspace* w, Job& J, RoundArgs& a, int budget, bool big, int nhub, int nchunk, KTimer& T) {
    hipStream_t st = w->stream;
    a.dev_plan = 1;
    wake_shape(a, J.n, budget);
    const int pgrid = std::max(std::min(nchunk, budget), 1);
    if (!w->ctl_h2) {
        if (hipHostMalloc(&w->ctl_h2, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return CSRCOLOR_ENOMEM;
        for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreateWithFlags(&w->pev[i], hipEventDisableTiming));
    }
    Ctl* mir[2] = {w->ctl_h, w->ctl_h2};
    long long rend[2] = {0, 0};
    int par = 1;             // parity of the worklists of the next round
    long long r = 2;         // next round (round 1 was k_round1)
    int k = 2;
    // batches of k rounds; the control block after batch b is copied back behind it and
    // read while batch b+1 runs, so the stream never waits for the host
    for (int b = 0;; ++b) {
        for (int i = 0; i < k; ++i) {
            a.par_in = par;
            a.par_out = par ^ 1;
            a.wl_in = w->wl[par];
            a.wl_out = w->wl[par ^ 1];
            a.wround = (int)r;
            if (a.ubytes) T.kern(1, k_wassign<true>, a.gdense, WG, a);
            else T.kern(1, k_wassign<false>, a.gdense, WG, a);
            if (a.ubytes) T.kern(2, k_detect_flags<true>, a.gdense, WG, a);
            else T.kern(2, k_detect_flags<false>, a.gdense, WG, a);
            // the worklists of the long rows, if any, in a launch of their own
            if (big) T.kern(2, k_detect<true>, detect_grid(w->device, budget), WG, a);
            if (nhub > 0) T.kern(2, k_push<true>, pgrid, WG, a);
            par ^= 1;
            ++r;
        }
        HIP_TRY(hipGetLastError());
        rend[b & 1] = r - 1;
        HIP_TRY(hipMemcpyAsync(mir[b & 1], w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(w->pev[b & 1], st));
        if (b > 0) {
            const int p = (b - 1) & 1;
            HIP_TRY(hipEventSynchronize(w->pev[p]));
            if (mir[p]->err) {
                (void)hipStreamSynchronize(st);
                return CSRCOLOR_EHIP;
            }
            if (mir[p]->rounds < rend[p]) break;    // the batch in flight only finds empty flags
            if (rend[p] > (long long)J.n + 2) {      // a colouring takes at most n rounds
                (void)hipStreamSynchronize(st);
                return CSRCOLOR_ELIMIT;
            }
        }
        k = std::min(k * 2, J.opt.sync_every);
    }
    return CSRCOLOR_OK;
}

// Graph mode: two rounds (parity 1 -> 0 -> 1) with device-side partitions are captured
// once into a hipGraph on a private stream and replayed; the queue sizes are read
// back every few replays.  The capture is reused while the kernel arguments stay the
// same (same arrays, sizes and options).
int drive_graph(Workspace* w, Job& J, RoundArgs& a, int budget) {
    a.dev_plan = 1;
    a.lbs_n = budget;
    if (!w->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&w->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&w->gev, hipEventDisableTiming));
    }
    const bool reuse = w->gexec && w->gbudget == budget && memcmp(&w->gargs, &a, sizeof(a)) == 0;
    if (!reuse) {
        if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
        w->gexec = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(w->gstream, hipStreamCaptureModeThreadLocal));
        RoundArgs r = a;
        for (int par = 1, i = 0; i < 2; ++i, par ^= 1) {
            r.par_in = par;
            r.par_out = par ^ 1;
            r.wl_in = w->wl[par];
            r.wl_out = w->wl[par ^ 1];
            k_assign<<<budget, WG, 0, w->gstream>>>(r);
            k_detect<false><<<detect_grid(w->device, budget), WG, 0, w->gstream>>>(r);
            if (r.pushff && r.cstart[1] != r.cstart[0]) k_push<false><<<budget, WG, 0, w->gstream>>>(r);  // split hubs exist
        }
        hipError_t ce = hipStreamEndCapture(w->gstream, &g);
        if (ce != hipSuccess) return CSRCOLOR_EHIP;
        ce = hipGraphInstantiate(&w->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ce != hipSuccess) {
            w->gexec = nullptr;
            return CSRCOLOR_EHIP;
        }
        w->gargs = a;
        w->gbudget = budget;
    }
    if (!w->ctl_h2) {
        if (hipHostMalloc(&w->ctl_h2, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return CSRCOLOR_ENOMEM;
        for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreateWithFlags(&w->pev[i], hipEventDisableTiming));
    }
    // the private stream waits for setup and round 1 on the caller's stream
    HIP_TRY(hipEventRecord(w->gev, w->stream));
    HIP_TRY(hipStreamWaitEvent(w->gstream, w->gev, 0));
    // batches of k replays, each read back one batch behind (rounds replayed past the end
    // find empty queues and do nothing), so the GPU never waits for the host
    Ctl* mir[2] = {w->ctl_h, w->ctl_h2};
    long long rend[2] = {0, 0};
    long long launched = 1;
    int k = 1;
    int rc = CSRCOLOR_OK;
    for (int b = 0;; ++b) {
        for (int i = 0; i < k; ++i) HIP_TRY(hipGraphLaunch(w->gexec, w->gstream));
        launched += 2 * k;
        rend[b & 1] = launched;
        HIP_TRY(hipMemcpyAsync(mir[b & 1], w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, w->gstream));
        HIP_TRY(hipEventRecord(w->pev[b & 1], w->gstream));
        if (b > 0) {
            const int p = (b - 1) & 1;
            HIP_TRY(hipEventSynchronize(w->pev[p]));
            if (mir[p]->err) {
                rc = CSRCOLOR_EHIP;
                break;
            }
            long long left = 0;
            for (int q = 0; q < NB; ++q) left += mir[p]->cnt[1][q];
            if (left == 0) break;
            if (rend[p] > (long long)J.n + 2) {
                rc = CSRCOLOR_ELIMIT;
                break;
            }
        }
        k = std::min(k * 2, std::max(1, J.opt.sync_every / 2));
    }
    HIP_TRY(hipStreamSynchronize(w->gstream));
    return rc;
}

// Graph mode with wake flags: two rounds (parity 1 -> 0 -> 1) of the launches drive_wake
// makes for a round, the round number kept on the device (the recolouring FirstFit
// advances it, the kernels after it read it), captured once into a hipGraph on a private
// stream and replayed; the control block is read back every few
// replays, and the run ends once a round has tested no vertex (rounds after it return
// at once).  The capture is reused while the kernel arguments stay the same.
int drive_wake_graph(Workspace* w, Job& J, RoundArgs& a, int budget, bool big, int nhub, int nchunk) {
    a.dev_plan = 1;
    a.lbs_n = budget;
    a.wround = 0;
    a.wround_dev = &w->ctl->wr;
    wake_shape(a, J.n, budget);
    const int pgrid = std::max(std::min(nchunk, budget), 1);
    if (!w->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&w->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&w->gev, hipEventDisableTiming));
    }
    const bool reuse = w->gexec && w->gbudget == budget && memcmp(&w->gargs, &a, sizeof(a)) == 0;
    if (!reuse) {
        if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
        w->gexec = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(w->gstream, hipStreamCaptureModeThreadLocal));
        RoundArgs r = a;
        for (int par = 1, i = 0; i < 2; ++i, par ^= 1) {
            r.par_in = par;
            r.par_out = par ^ 1;
            r.wl_in = w->wl[par];
            r.wl_out = w->wl[par ^ 1];
            k_wassign<false><<<a.gdense, WG, 0, w->gstream>>>(r);
            k_detect_flags<false><<<a.gdense, WG, 0, w->gstream>>>(r);
            if (big) k_detect<true><<<detect_grid(w->device, budget), WG, 0, w->gstream>>>(r);
            if (nhub > 0) k_push<true><<<pgrid, WG, 0, w->gstream>>>(r);
        }
        hipError_t ce = hipStreamEndCapture(w->gstream, &g);
        if (ce != hipSuccess) return CSRCOLOR_EHIP;
        ce = hipGraphInstantiate(&w->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ce != hipSuccess) {
            w->gexec = nullptr;
            return CSRCOLOR_EHIP;
        }
        w->gargs = a;
        w->gbudget = budget;
    }
    if (!w->ctl_h2) {
        if (hipHostMalloc(&w->ctl_h2, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return CSRCOLOR_ENOMEM;
        for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreateWithFlags(&w->pev[i], hipEventDisableTiming));
    }
    // the private stream waits for setup and round 1 on the caller's stream
    HIP_TRY(hipEventRecord(w->gev, w->stream));
    HIP_TRY(hipStreamWaitEvent(w->gstream, w->gev, 0));
    // batches of k replays; the control block after batch b is copied back behind it and
    // read while batch b+1 runs (as in drive_wake), so the GPU never waits for the host
    Ctl* mir[2] = {w->ctl_h, w->ctl_h2};
    long long rend[2] = {0, 0};
    long long last = 1;      // the last round launched
    int k = 1;
    int rc = CSRCOLOR_OK;
    for (int b = 0;; ++b) {
        for (int i = 0; i < k; ++i) HIP_TRY(hipGraphLaunch(w->gexec, w->gstream));
        last += 2 * k;
        rend[b & 1] = last;
        HIP_TRY(hipMemcpyAsync(mir[b & 1], w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, w->gstream));
        HIP_TRY(hipEventRecord(w->pev[b & 1], w->gstream));
        if (b > 0) {
            const int p = (b - 1) & 1;
            HIP_TRY(hipEventSynchronize(w->pev[p]));
            if (mir[p]->err) {
                rc = CSRCOLOR_EHIP;
                break;
            }
            if (mir[p]->rounds < rend[p]) break;    // a round tested no vertex: all settled
            if (rend[p] > (long long)J.n + 2) {      // a colouring takes at most n rounds
                rc = CSRCOLOR_ELIMIT;
                break;
            }
        }
        k = std::min(k * 2, std::max(1, J.opt.sync_every / 2));
    }
    // the batch still in flight only finds a finished colouring
    HIP_TRY(hipStreamSynchronize(w->gstream));
    return rc;
}

// Topology-driven rounds: FirstFit and the conflict test over all n vertices; the
// loser count of the last enqueued round is read back every few rounds.
int drive_topo(Workspace* w, Job& J, int budget, int st_cap, KTimer& T) {
    hipStream_t st = w->stream;
    const int n = J.n;
    const int cus = num_cus(w->device);
    // X = 0 (every vertex uncoloured); "losers of round 0" = n, so round 1 is booked
    T.run(0, [&] {
        k_fill<<<std::min((n + WG - 1) / WG, cus * 8), WG, 0, st>>>(w->X, n, 0);
        k_fill<<<1, 64, 0, st>>>(&w->ctl->cnt[1][0], 1, n);
    });
    const int grid = (int)std::max<long long>(1, std::min<long long>(((long long)n + WG - 1) / WG, budget));
    long long* wsz = st_cap ? w->st_wsize : nullptr;
    int par = 0;
    long long launched = 0;
    int k = 2;
    for (;;) {
        for (int i = 0; i < k; ++i) {
            T.kern(1, k_topo_assign, grid, WG, n, J.rowptr, (const int*)J.colidx, w->X, w->ctl, par, wsz, st_cap);
            T.kern(2, k_topo_detect, grid, WG, n, J.rowptr, J.colidx, w->X, J.colors_out, w->ctl, par, J.sorted,
                   J.opt.rule);
            par ^= 1;
            ++launched;
        }
        HIP_TRY(hipGetLastError());
        int rc = read_ctl(w);
        if (rc) return rc;
        if (w->ctl_h->err) return CSRCOLOR_EHIP;
        if (w->ctl_h->cnt[par ^ 1][0] == 0) break;
        if (launched > (long long)n + 2) return CSRCOLOR_ELIMIT;
        k = std::min(k * 2, J.opt.sync_every);
    }
    return CSRCOLOR_OK;
}

// Worklist rounds (SGR and JP): split-row scratch, push bitmaps, round 1 (JP: the
// initial worklist), then the rounds in the requested drive mode.
int run_rounds(Workspace* w, Job& J, const int hist[NB], const Seg& seg, int st_cap, KTimer& T) {
    const int n = J.n;
    hipStream_t st = w->stream;
    const int cus = num_cus(w->device);
    const int twave = J.opt.twave;
    int rc = 0;
    // split-row scratch: cstart[2] (hubs), owner[2] (chunks), hub bitmaps, done counters, lost flags
    const int nhub = hist[BSPLIT];
    const int nchunk = w->ctl_h->hchunks;
    // live lists: the vertices of degree > 61 scan lists of their uncoloured lower
    // neighbours (id rule, worklist SGR only)
    const bool use_live = J.opt.live && J.opt.rule <= 1 && J.opt.algo == CSRCOLOR_ALGO_SGR &&
                          hist[NTILE] + hist[NTILE + 1] + hist[BSPLIT] > 0;
    // with live lists the chunk records come first (16-byte aligned)
    const size_t recs = use_live ? 8 * (size_t)nchunk : 0;
    const size_t split_ints = recs + 2 * (size_t)nhub + 2 * (size_t)nchunk + (size_t)nhub * (HW + 4) +
                              (use_live ? 2 * (size_t)nchunk : 0) + 2 * (size_t)nchunk;
    if ((rc = ensure_split(w, split_ints))) return rc;
    int4* crec0 = use_live ? reinterpret_cast<int4*>(w->split) : nullptr;
    int4* crec1 = use_live ? crec0 + nchunk : nullptr;
    int* cstart0 = w->split + recs;
    int* cstart1 = cstart0 + nhub;
    int* owner0 = cstart1 + nhub;
    int* owner1 = owner0 + nchunk;
    int* hubflags = owner1 + nchunk;   // HW bitmap words + done + lost + 64-bit merge word per hub
    if (nhub > 0) {
        const int cnt = nhub * (HW + 4);
        k_fill<<<std::min((cnt + WG - 1) / WG, cus * 4), WG, 0, st>>>(hubflags, cnt, 0);
    }
    int* clen = use_live ? hubflags + (size_t)nhub * (HW + 4) : nullptr;   // per-chunk live lengths
    int* cpos = use_live ? clen + nchunk : nullptr;                          // and resume positions
    int* settled = hubflags + (size_t)nhub * (HW + 4) + (use_live ? 2 * (size_t)nchunk : 0);
    if (use_live && (rc = ensure_live(w, std::max<size_t>((size_t)w->ctl_h->nnz, 1)))) return rc;

    // conflict hints and live lists serve both rules (a hint or list entry beat the vertex
    // when it was recorded, and ids and degrees never change); wake flags the id rule only
    int* hint = (J.opt.hints && J.opt.rule <= 1) ? w->hint : nullptr;
    // wake flags need the id rule's hints, push FirstFit and the host loop; ordered
    // compaction is a property of the full worklists they replace
    // auto: the sleeping vertices are the short ones; where long rows hold most arcs the
    // full worklist rounds measured faster (R-MAT: 66 vs 78 ms at scale 23)
    const bool wake_wanted = J.opt.wake > 0 || (J.opt.wake == 0 && w->ctl_h->bigarcs * 10 < w->ctl_h->nnz);
    // (colour words keep BIG at bit 30, so colours must stay below 2^30)
    const bool use_wake = wake_wanted && hint && J.opt.rule == 0 && J.opt.pushff && J.opt.algo == CSRCOLOR_ALGO_SGR &&
                          (J.opt.mode == CSRCOLOR_MODE_LOOP ||
                           (J.opt.mode == CSRCOLOR_MODE_GRAPH && !(J.stats && J.stats->kernel_bytes))) &&
                          !J.opt.ordered && J.maxdeg < CMASK - 1;
    const bool longrows = hist[NTILE] + hist[NTILE + 1] + hist[BSPLIT] > 0;
    J.wake = use_wake;
    if (use_wake) {
        const int fw = (int)(flag_bytes((size_t)n) / 4);
        T.run(0, [&] {
            k_fill<<<std::min((fw + WG - 1) / WG, cus * 8), WG, 0, st>>>(reinterpret_cast<int*>(w->rflag), fw, 0);
            k_fill<<<std::min((fw + WG - 1) / WG, cus * 8), WG, 0, st>>>(reinterpret_cast<int*>(w->aflag), fw, 0);
            for (size_t off = 0; off < 2 * (size_t)n; off += (size_t)1 << 30) {
                const int cnt = (int)std::min<size_t>(2 * (size_t)n - off, (size_t)1 << 30);
                k_fill<<<std::min((cnt + WG - 1) / WG, cus * 8), WG, 0, st>>>(reinterpret_cast<int*>(w->Fs) + off,
                                                                                cnt, 0);
            }
        });
    }

    // push mode: deg(v)+1 bits per vertex, zeroed
    unsigned* F = nullptr;
    if (J.opt.pushff) {
        // one flag per (vertex, colour <= deg+1): bits, or bytes
        const size_t flags = (size_t)w->ctl_h->nnz + (size_t)n;
        const size_t words = J.opt.pushff == 2 ? flags / 4 + 4 : flags / 32 + 2;
        if ((rc = ensure_F(w, words))) return rc;
        F = w->F;
        // with wake flags only the long rows use these flags (short ones: Fs)
        if (!use_wake || longrows) {
            T.run(0, [&] {
                k_fill<<<(int)std::min<size_t>((words + WG - 1) / WG, (size_t)cus * 8), WG, 0, st>>>(
                    reinterpret_cast<int*>(F), (int)words, 0);
            });
        }
        const int dwords = n / 4 + 1;
        if (!use_wake) {
            T.run(0, [&] {
                k_fill<<<std::min((dwords + WG - 1) / WG, cus * 8), WG, 0, st>>>(reinterpret_cast<int*>(w->dirty),
                                                                                    dwords, 0);
                if (J.opt.pushff == 2) {
                    // the small-colour flag slots, KQ bytes per vertex
                    const size_t qw = (size_t)n * (KQ / 4);
                    for (size_t off = 0; off < qw; off += (size_t)1 << 30) {
                        const int cnt = (int)std::min<size_t>(qw - off, (size_t)1 << 30);
                        k_fill<<<std::min((cnt + WG - 1) / WG, cus * 8), WG, 0, st>>>(
                            reinterpret_cast<int*>(w->Fq) + off, cnt, 0);
                    }
                }
            });
        }
    }
    const int r1blocks = (int)(((long long)n + 4 * WG - 1) / (4 * WG));
    // ordered compaction: look-back status words, NB per round-1 block, then one per
    // block of the largest round grid (cleared before each use)
    const int budget = cus * J.opt.blocks_per_cu;
    const size_t lb_round = (size_t)budget + 2 * NB + (size_t)n / SUB + 8;
    unsigned long long* lb = nullptr;
    if (J.opt.ordered) {
        if ((rc = ensure_lb(w, std::max((size_t)NB * r1blocks, lb_round)))) return rc;
        lb = w->lb;
        const size_t ints = 2 * (size_t)NB * r1blocks;
        T.run(0, [&] {
            k_fill<<<(int)std::min<size_t>((ints + WG - 1) / WG, (size_t)cus * 8), WG, 0, st>>>(
                reinterpret_cast<int*>(lb), (int)ints, 0);
        });
    }
    T.run(0, [&] {
        k_round1<<<r1blocks, WG, 0, st>>>(n, J.rowptr, J.colidx, w->X, J.colors_out, w->wl[1], w->ctl,
                                          J.sorted, twave, J.opt.tsplit, seg, cstart1, owner1, F,
                                          w->ctl_h->nnz, J.opt.rule, J.opt.algo == CSRCOLOR_ALGO_JP, hint,
                                          use_live ? w->llen : nullptr, clen, lb, J.opt.pushff == 2,
                                          (F && !use_wake) ? w->dirty : nullptr,
                                          use_wake ? w->rflag : nullptr, w->aflag, use_wake ? w->srnd : nullptr,
                                          w->Fs, (J.opt.pushff == 2 && !use_wake) ? w->Fq : nullptr, crec1,
                                          J.opt.tiles);
    });
    HIP_TRY(hipGetLastError());

    RoundArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.rowptr = J.rowptr;
    a.colidx = J.colidx;
    a.X = w->X;
    a.out = J.colors_out;
    a.ctl = w->ctl;
    a.twave = twave;
    a.tiles = J.opt.tiles;
    a.sorted = J.sorted;
    a.nnz = w->ctl_h->nnz;
    a.lane_mode_assign = J.opt.lane_assign;
    a.lane_mode_detect = J.opt.lane_detect;
    a.tsplit = J.opt.tsplit;
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
    a.settled = (J.opt.pushff && nhub > 0) ? settled : nullptr;
    a.settled_k = settled + nchunk;
    a.pushff = J.opt.pushff;
    a.F = F;
    a.dirty = (F && !use_wake) ? w->dirty : nullptr;
    a.Fq = (J.opt.pushff == 2 && !use_wake) ? w->Fq : nullptr;
    if (use_wake) {
        a.rflag = w->rflag;
        a.aflag = w->aflag;
        a.srnd = w->srnd;
        a.hflag = FLAG;
        a.Fs = w->Fs;
        if (J.stats && J.stats->kernel_bytes) {
            k_fill<<<1, 64, 0, st>>>(reinterpret_cast<int*>(w->ubytes), 4, 0);
            a.ubytes = w->ubytes;
        }
    }
    a.rule = J.opt.rule;
    a.seed = J.opt.seed;
    a.hint = hint;
    a.lbs = lb;
    a.live = use_live ? w->live : nullptr;
    a.llen = use_live ? w->llen : nullptr;
    a.clen = clen;
    a.lpos = use_live ? w->lpos : nullptr;
    a.cpos = cpos;
    a.st_cap = st_cap;
    a.st_wsize = st_cap ? w->st_wsize : nullptr;
    a.st_arcs = st_cap ? w->st_arcs : nullptr;
    for (int b = 0; b <= NB; ++b) a.seg[b] = seg.s[b];
    if (st_cap) {
        HIP_TRY(hipMemsetAsync(w->st_wsize, 0, st_cap * sizeof(long long), st));
        HIP_TRY(hipMemsetAsync(w->st_arcs, 0, st_cap * sizeof(long long), st));
    }

    if (J.opt.mode == CSRCOLOR_MODE_GRAPH) {
        rc = use_wake ? drive_wake_graph(w, J, a, budget, longrows, nhub, nchunk) : drive_graph(w, J, a, budget);
    } else if (use_wake) {
        rc = drive_wake(w, J, a, budget, longrows, nhub, nchunk, T);
    } else {
        int ub[NB];
        for (int b = 0; b < NB; ++b) ub[b] = hist[b];
        ub[BSPLIT] = nchunk;
        rc = drive_loop(w, J, a, ub, budget, T);
    }
    return rc;
}

// After the rounds: per-round statistics rebuilt from settling rounds (wake flags), the
// colour count and the statistics the caller asked for.
int finish_job(Workspace* w, Job& J, int st_cap, KTimer& T, int vblocks) {
    const int n = J.n;
    hipStream_t st = w->stream;
    int rc = 0;
    if (J.wake && st_cap) {
        // per-round settle counts and their arcs, from the settling rounds
        k_round_hist<<<std::max(vblocks, 1), WG, 0, st>>>(n, J.rowptr, w->srnd, w->st_wsize, w->st_arcs, st_cap);
        HIP_TRY(hipGetLastError());
    }
    if ((rc = read_ctl(w))) return rc;
    // Vertex 0 has no lower neighbour, so it always settles in round 1 with colour 1
    // (round-1 winners do not touch the device maximum).
    J.ncolors = std::max(w->ctl_h->maxcolor, 1);
    J.rounds = std::max(w->ctl_h->rounds, 1);
    J.nnz = w->ctl_h->nnz;
    if (J.stats) {
        J.stats->nnz = J.nnz;
        if (T.on) {
            J.stats->ms_setup = T.total_ms(0, nullptr);
            J.stats->ms_assign = T.total_ms(1, &J.stats->n_assign);
            J.stats->ms_detect = T.total_ms(2, &J.stats->n_detect);
        } else {
            J.stats->ms_setup = J.stats->ms_assign = J.stats->ms_detect = 0;
            J.stats->n_assign = J.stats->n_detect = 0;
        }
        if (J.stats->kernel_bytes) {
            J.stats->kernel_bytes[0] = J.stats->kernel_bytes[1] = 0;
            if (J.wake) {
                unsigned long long kb[2];
                HIP_TRY(hipMemcpyAsync(kb, w->ubytes, sizeof(kb), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                J.stats->kernel_bytes[0] = (int64_t)kb[0];
                J.stats->kernel_bytes[1] = (int64_t)kb[1];
            }
        }
        J.stats->rounds = J.rounds;
        J.stats->ncolors = J.ncolors;
        J.stats->rows_sorted = J.sorted;
        J.stats->max_degree = J.maxdeg;
        const int m = std::min(J.rounds, st_cap);
        if (m > 0) {
            std::vector<long long> tmp(m);
            if (J.stats->wsize) {
                HIP_TRY(hipMemcpyAsync(tmp.data(), w->st_wsize, m * sizeof(long long), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (J.wake) {
                    // tmp[r]: vertices settled in round r+1; W_1 = V
                    long long left = n;
                    for (int r = 0; r < m; ++r) {
                        J.stats->wsize[r] = left;
                        left -= tmp[r];
                    }
                } else {
                    for (int r = 0; r < m; ++r) J.stats->wsize[r] = tmp[r];
                }
                J.stats->wsize[0] = n;
            }
            if (J.stats->arcs) {
                HIP_TRY(hipMemcpyAsync(tmp.data(), w->st_arcs, m * sizeof(long long), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (J.wake) {
                    long long left = w->ctl_h->nnz;
                    for (int r = 0; r < m; ++r) {
                        J.stats->arcs[r] = left;
                        left -= tmp[r];
                    }
                } else {
                    for (int r = 0; r < m; ++r) J.stats->arcs[r] = tmp[r];
                }
                J.stats->arcs[0] = w->ctl_h->nnz;
            }
        }
    }
    return CSRCOLOR_OK;
}


// Status of a device-planned run from its control block (the host twin of dev_status).
int status_of(const Ctl* c) {
    const int e = c->err;
    if (e & (ERR_ROWPTR | ERR_COLIDX | ERR_MULTI | ERR_BATCH)) return CSRCOLOR_EBADCSR;
    if (e & ERR_ASYM) return CSRCOLOR_ENOTSYM;
    if (e & ERR_UNSORTED) return CSRCOLOR_EINVAL;
    if (e & ERR_NOMEM) return CSRCOLOR_ENOMEM;
    if (e & ERR_BARRIER) return CSRCOLOR_ETIMEOUT;
    if (e) return CSRCOLOR_EHIP;
    if (!c->pdone) return CSRCOLOR_ELIMIT;
    return CSRCOLOR_OK;
}

int g_pers_per_cu[64] = {0};
long long g_wall_khz[64] = {0};

// Workgroups of the persistent round kernel: no more than fit on the device at once
// (every barrier waits for all of them), no more than the launch budget, and for
// small graphs about one per 256 vertices (fewer blocks make every barrier cheaper).
int persistent_grid(int dev, int n, int budget) {
    if (dev < 0 || dev >= 64) dev = 0;
    if (g_pers_per_cu[dev] == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_persistent_dev, WG, 0) !=
                hipSuccess || per_cu <= 0)
            per_cu = 1;
        g_pers_per_cu[dev] = per_cu;
    }
    const int resident = g_pers_per_cu[dev] * num_cus(dev);
    const int want = (int)std::max<long long>(64, ((long long)n + 255) / 256);
    return std::max(std::min(std::min(resident, budget), want), std::min(resident, 16));
}

// Wall-clock ticks a persistent barrier may wait before giving up (8 seconds).
long long barrier_limit(int dev) {
    if (dev < 0 || dev >= 64) dev = 0;
    if (g_wall_khz[dev] == 0) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        g_wall_khz[dev] = khz;
    }
    return 8000LL * g_wall_khz[dev];
}

// Launches of a device-planned run over a workspace whose buffers are already sized
// (every size the kernels rely on is checked again on the device by the plan kernel).
// `plain` launches the persistent round kernel as an ordinary kernel of no more
// workgroups than fit on the device at once (for stream capture and for the
// allocation-free entry point; its barriers are bounded, so a grid that is not
// resident ends with CSRCOLOR_ETIMEOUT), else cooperatively.  Makes no allocation,
// no copy and no wait.
int enqueue_device(Workspace* w, Job& J, const long long* voff, int G, int* ncolors_dev, KTimer& T, bool plain,
                   int* vblocks_out) {
    const int n = J.n;
    hipStream_t st = w->stream;
    const Options& o = J.opt;
    const int st_cap = J.stats ? std::max(J.stats->cap, 0) : 0;
    const int cus = num_cus(w->device);
    const int budget = cus * o.blocks_per_cu;
    const int grid = persistent_grid(w->device, n, budget);
    const int r1blocks = (int)(((long long)n + 4 * WG - 1) / (4 * WG));
    unsigned long long* lb = nullptr;
    if (o.ordered) {
        if (!w->lb || w->lb_cap < std::max((size_t)NB * r1blocks, (size_t)grid + 2 * NB + 8)) return CSRCOLOR_EINVAL;
        lb = w->lb;
    }

    RoundArgs t;
    memset(&t, 0, sizeof(t));
    t.n = n;
    t.rowptr = J.rowptr;
    t.colidx = J.colidx;
    t.X = w->X;
    t.out = J.colors_out;
    t.ctl = w->ctl;
    t.wl_in = w->wl[1];
    t.wl_out = w->wl[0];
    t.twave = o.twave;
    t.tiles = o.tiles;
    t.tsplit = o.tsplit;
    t.lane_mode_assign = o.lane_assign;
    t.lane_mode_detect = o.lane_detect;
    t.dev_plan = 1;
    t.pushff = o.pushff;
    t.F = w->F;
    t.dirty = w->dirty;
    t.rule = o.rule;
    t.hint = (o.hints && o.rule <= 1) ? w->hint : nullptr;
    t.live = w->live;
    t.llen = w->llen;
    t.lpos = w->lpos;
    t.Fq = w->Fq;
    t.lbs = lb;
    t.lbs_n = grid;
    t.st_cap = st_cap;
    t.st_wsize = st_cap ? w->st_wsize : nullptr;
    t.st_arcs = st_cap ? w->st_arcs : nullptr;
    DevCaps c;
    c.f_words = (long long)w->F_cap;
    c.live_ints = (long long)w->live_cap;
    c.split_ints = (long long)w->split_cap;
    c.split = w->split;
    c.lb1 = lb;
    c.lb1_ints = lb ? 2 * NB * r1blocks : 0;
    c.want_live = o.live && o.rule <= 1 && w->live != nullptr;

    T.run(0, [&] { k_init<<<1, WG, 0, st>>>(w->ctl); });
    const int vblocks = (int)std::min<long long>(((long long)n + WG - 1) / WG, (long long)cus * 4);
    if (vblocks_out) *vblocks_out = vblocks;
    const int rblocks = (int)std::max<long long>(
        1, std::min<long long>(((long long)n + WG * VROWS - 1) / (WG * VROWS), (long long)cus * 4));
    T.kern(0, k_validate_rows, rblocks, WG, n, J.rowptr, J.colidx, w->ctl, o.twave, o.tsplit, J.expect_nnz,
           o.tiles);
    T.kern(0, k_validate_arcs, cus * 4, WG, n, J.rowptr, J.colidx, w->ctl);
    if (voff) k_validate_batch<<<cus * 4, WG, 0, st>>>(G, n, voff, J.rowptr, J.colidx, w->ctl);
    if (o.validate >= 1) k_check_symmetric<<<std::max(vblocks, 1), WG, 0, st>>>(n, J.rowptr, J.colidx, w->ctl);
    if (st_cap) {
        k_fill<<<std::max(1, std::min((2 * st_cap + WG - 1) / WG, cus)), WG, 0, st>>>(
            reinterpret_cast<int*>(w->st_wsize), 2 * st_cap, 0);
        k_fill<<<std::max(1, std::min((2 * st_cap + WG - 1) / WG, cus)), WG, 0, st>>>(
            reinterpret_cast<int*>(w->st_arcs), 2 * st_cap, 0);
    }
    T.run(0, [&] {
        k_dev_plan<<<1, 64, 0, st>>>(t, c, w->plan);
        k_dev_clear<<<cus * 4, WG, 0, st>>>(w->plan);
        k_round1_dev<<<std::max(r1blocks, 1), WG, 0, st>>>(w->plan);
    });
    HIP_TRY(hipGetLastError());
    const DevPlan* plan = w->plan;
    int maxr = n + 2;
    long long limit = barrier_limit(w->device);
    hipError_t e = hipSuccess;
    T.run(1, [&] {
        if (plain) {
            k_persistent_dev<<<grid, WG, 0, st>>>(plan, maxr, limit);
            e = hipGetLastError();
        } else {
            void* args[] = {&plan, &maxr, &limit};
            e = hipLaunchCooperativeKernel((const void*)k_persistent_dev, dim3(grid), dim3(WG), args, 0, st);
        }
    });
    HIP_TRY(e);
    if (ncolors_dev) {
        const int fg = G > 0 ? std::min(G, cus * 8) : 1;
        k_dev_finish<<<fg, WG, 0, st>>>(w->ctl, G, voff, J.colors_out, ncolors_dev);
        HIP_TRY(hipGetLastError());
    }
    return CSRCOLOR_OK;
}

// Device-planned run (the rounds of Sec. 3.1 driven on the device, see sgr_plan.h):
// everything is enqueued on the workspace stream.  The arc-sized buffers (push flags,
// live lists, split-row scratch) are sized on the host from a read-back of rowptr[n]
// when the call is synchronous (`sync`) or the workspace has never been sized for this
// many vertices; otherwise the call makes no allocation, no copy and no wait, and the
// plan kernel checks that the graph fits (ERR_NOMEM when it does not).  With `sync`
// the call waits and fills J (colour count, rounds, statistics) or returns the status
// the device found; `ncolors_dev` (device, may be null) receives the colour count, or
// for G > 0 graphs one count per graph, or the negative status.
int run_device(Workspace* w, Job& J, const long long* voff, int G, int* ncolors_dev, bool sync) {
    const int n = J.n;
    hipStream_t st = w->stream;
    const Options& o = J.opt;
    const int st_cap = J.stats ? std::max(J.stats->cap, 0) : 0;
    // the arc-sized buffers must cover every graph of at most cap_n vertices and arc_cap
    // arcs (a host-driven call may have grown the vertex arrays since they were sized)
    const bool covered = w->arc_cap > 0 && w->F_cap >= (w->cap_n + (size_t)w->arc_cap) / 4 + 4 &&
                         w->split_cap >= (size_t)(w->arc_cap / 16 + 64) && w->live_cap >= (size_t)w->arc_cap;
    const bool fresh = (size_t)n > w->cap_n || !w->ctl || !w->plan || !covered;
    int rc = ensure_capacity(w, (size_t)n, st_cap);
    if (rc) return rc;
    if (!w->plan && hipMalloc(&w->plan, sizeof(DevPlan)) != hipSuccess) return CSRCOLOR_ENOMEM;
    if (!w->sz_h && hipHostMalloc(&w->sz_h, sizeof(int), hipHostMallocDefault) != hipSuccess) return CSRCOLOR_ENOMEM;
    if (sync || fresh) {
        HIP_TRY(hipMemcpyAsync(w->sz_h, J.rowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const long long arcs = std::max<long long>(std::max(*w->sz_h, 0), w->arc_cap);
        // byte flags for every vertex and arc the workspace holds (the larger flag
        // variant); split-row scratch for the most hubs and chunks that many arcs allow
        // (a hub has more than 1024 arcs: 38 ints per hub, 14 per 2048-arc chunk)
        if ((rc = ensure_F(w, (size_t)((w->cap_n + arcs) / 4 + 4)))) return rc;
        if ((rc = ensure_split(w, (size_t)(arcs / 16 + 64)))) return rc;
        if ((rc = ensure_live(w, (size_t)std::max<long long>(arcs, 1)))) return rc;
        w->arc_cap = std::max<long long>(arcs, 1);
    }
    if (o.ordered) {
        const int cus = num_cus(w->device);
        const int grid = persistent_grid(w->device, n, cus * o.blocks_per_cu);
        const int r1blocks = (int)(((long long)n + 4 * WG - 1) / (4 * WG));
        if ((rc = ensure_lb(w, std::max((size_t)NB * r1blocks, (size_t)grid + 2 * NB + 8)))) return rc;
    }
    // every later round in one launch: cooperative (the runtime guarantees that every
    // workgroup is resident) unless the stream is being captured into a graph
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
    KTimer T(w, J.stats && J.stats->time_kernels);
    int vblocks = 0;
    if ((rc = enqueue_device(w, J, voff, G, ncolors_dev, T, cs == hipStreamCaptureStatusActive, &vblocks))) return rc;
    if (!sync) return CSRCOLOR_OK;
    if ((rc = read_ctl(w))) return rc;
    if ((rc = status_of(w->ctl_h))) return rc;
    J.sorted = w->ctl_h->desc_total == w->ctl_h->desc_bound;
    J.maxdeg = w->ctl_h->maxdeg;
    J.wake = false;
    return finish_job(w, J, st_cap, T, vblocks);
}

int run_job(Workspace* w, Job& J, const long long* voff, int G) {
    if (J.opt.mode == CSRCOLOR_MODE_PERSISTENT) return run_device(w, J, voff, G, nullptr, true);
    const int n = J.n;
    hipStream_t st = w->stream;
    const int st_cap = J.stats ? std::max(J.stats->cap, 0) : 0;
    int rc = ensure_capacity(w, (size_t)n, st_cap);
    if (rc) return rc;
    const int cus = num_cus(w->device);
    const int twave = J.opt.twave;

    KTimer T(w, J.stats && J.stats->time_kernels);
    T.run(0, [&] { k_init<<<1, WG, 0, st>>>(w->ctl); });
    const int vblocks = (int)std::min<long long>(((long long)n + WG - 1) / WG, (long long)cus * 4);
    const int rblocks = (int)std::max<long long>(
        1, std::min<long long>(((long long)n + WG * VROWS - 1) / (WG * VROWS), (long long)cus * 4));
    T.kern(0, k_validate_rows, rblocks, WG, n, J.rowptr, J.colidx, w->ctl, twave, J.opt.tsplit, -1LL,
           J.opt.tiles);
    // the arc pass skips itself when the vertex pass found an error, so one read-back
    // covers both
    T.kern(0, k_validate_arcs, cus * 4, WG, n, J.rowptr, J.colidx, w->ctl);
    if (voff) k_validate_batch<<<cus * 4, WG, 0, st>>>(G, n, voff, J.rowptr, J.colidx, w->ctl);
    HIP_TRY(hipGetLastError());
    if ((rc = read_ctl(w))) return rc;
    if (w->ctl_h->err) return CSRCOLOR_EBADCSR;
    J.sorted = w->ctl_h->desc_total == w->ctl_h->desc_bound;
    J.maxdeg = w->ctl_h->maxdeg;
    if (J.opt.validate >= 1) {
        if (!J.sorted) return CSRCOLOR_EINVAL;   // symmetry check needs sorted rows
        k_check_symmetric<<<vblocks, WG, 0, st>>>(n, J.rowptr, J.colidx, w->ctl);
        HIP_TRY(hipGetLastError());
        if ((rc = read_ctl(w))) return rc;
        if (w->ctl_h->err & 4) return CSRCOLOR_ENOTSYM;
        if (w->ctl_h->err) return CSRCOLOR_EBADCSR;
    }
    int hist[NB];
    Seg seg;
    seg.s[0] = 0;
    for (int b = 0; b < NB; ++b) {
        hist[b] = w->ctl_h->hist[b];
        seg.s[b + 1] = seg.s[b] + hist[b];
    }

    if (J.opt.algo == CSRCOLOR_ALGO_SGR_TOPO) {
        if (st_cap) HIP_TRY(hipMemsetAsync(w->st_wsize, 0, st_cap * sizeof(long long), st));
        if (st_cap) HIP_TRY(hipMemsetAsync(w->st_arcs, 0, st_cap * sizeof(long long), st));
        rc = drive_topo(w, J, cus * J.opt.blocks_per_cu, st_cap, T);
    } else {
        rc = run_rounds(w, J, hist, seg, st_cap, T);
    }
    if (rc) return rc;
    return finish_job(w, J, st_cap, T, vblocks);
}

// ---------------------------------------------------------------------------
// Allocation-free colouring (csrcolor_color_noalloc): the device-planned run over a
// fixed scratch array in the library's own device memory, for callers that cannot
// allocate.  Layout (byte offsets, each part 256-byte aligned): control block, plan
// block, colour state, two worklists, conflict hints, live-list lengths (split rows'
// chunk bases), live-list resume positions, dirty bytes, small-colour flag slots, byte
// flags of the forbidden colours for every vertex and arc, split-row scratch.  Live
// lists are off (they would need 4 bytes per arc more).
// ---------------------------------------------------------------------------
constexpr size_t na_align(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t NA_N = CSRCOLOR_NOALLOC_MAX_N;
constexpr size_t NA_E = CSRCOLOR_NOALLOC_MAX_NNZ;
constexpr size_t NA_F_WORDS = (NA_N + NA_E) / 4 + 4;
constexpr size_t NA_SPLIT_INTS = NA_E / 21 + 64;   // without live lists: 38 ints per hub, 4 per chunk
constexpr size_t NA_CTL = 0;
constexpr size_t NA_PLAN = na_align(sizeof(Ctl));
constexpr size_t NA_X = NA_PLAN + na_align(sizeof(DevPlan));
constexpr size_t NA_WL0 = NA_X + na_align(4 * NA_N);
constexpr size_t NA_WL1 = NA_WL0 + na_align(4 * NA_N);
constexpr size_t NA_HINT = NA_WL1 + na_align(4 * NA_N);
constexpr size_t NA_LLEN = NA_HINT + na_align(4 * NA_N);
constexpr size_t NA_LPOS = NA_LLEN + na_align(4 * NA_N);
constexpr size_t NA_DIRTY = NA_LPOS + na_align(4 * NA_N);
constexpr size_t NA_FQ = NA_DIRTY + na_align(NA_N + 16);
constexpr size_t NA_F = NA_FQ + na_align(KQ * NA_N);
constexpr size_t NA_SPLIT = NA_F + na_align(4 * NA_F_WORDS);
constexpr size_t NA_BYTES = NA_SPLIT + na_align(4 * NA_SPLIT_INTS);
static_assert(NA_BYTES <= ((size_t)CSRCOLOR_NOALLOC_SCRATCH_MIB << 20), "scratch layout exceeds its stated size");

// One copy per device, held from the code object's load until the process ends.  In
// host code this name is only a stand-in for the symbol: kernels receive the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

struct NoAllocDev {
    bool ready = false;
    unsigned char* ptr = nullptr;   // this device's address of `scratch`
    Workspace ws;                   // views into it; never freed
};
NoAllocDev g_na[64];
std::mutex g_na_mu;

// The workspace of the allocation-free entry point on device `dev` (the current
// device): on the first call, looks up this device's address of the scratch array
// and lays the buffers out in it.
Workspace* noalloc_ws(int dev, int* rc) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    NoAllocDev& d = g_na[dev];
    if (!d.ready) {
        unsigned char* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            *rc = CSRCOLOR_EHIP;
            return nullptr;
        }
        Workspace& w = d.ws;
        w.device = dev;
        w.cap_n = NA_N;
        w.ctl = reinterpret_cast<Ctl*>(ptr + NA_CTL);
        w.plan = reinterpret_cast<DevPlan*>(ptr + NA_PLAN);
        w.X = reinterpret_cast<int*>(ptr + NA_X);
        w.wl[0] = reinterpret_cast<int*>(ptr + NA_WL0);
        w.wl[1] = reinterpret_cast<int*>(ptr + NA_WL1);
        w.hint = reinterpret_cast<int*>(ptr + NA_HINT);
        w.llen = reinterpret_cast<int*>(ptr + NA_LLEN);
        w.lpos = reinterpret_cast<int*>(ptr + NA_LPOS);
        w.dirty = ptr + NA_DIRTY;
        w.Fq = ptr + NA_FQ;
        w.F = reinterpret_cast<unsigned*>(ptr + NA_F);
        w.F_cap = NA_F_WORDS;
        w.split = reinterpret_cast<int*>(ptr + NA_SPLIT);
        w.split_cap = NA_SPLIT_INTS;
        w.live = nullptr;
        w.live_cap = 0;
        w.arc_cap = (long long)NA_E;
        d.ptr = ptr;
        d.ready = true;
    }
    return &d.ws;
}

}  // namespace
}  // namespace csrcolor

using namespace csrcolor;

extern "C" {

}  // extern "C"

namespace {
// Host-driven colouring of one graph (every mode but the device-planned one): the call
// waits for the stream and returns the colour count on the host.
int color_host(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* colors_out,
               int32_t* ncolors_host, const csrcolor_opts* opts, csrcolor_stats* stats, hipStream_t stream) {
    if (n < 0) return CSRCOLOR_EINVAL;
    if (!opts_valid(opts, true)) return CSRCOLOR_EINVAL;
    if (stats && stats->cap > 0 && stats->cap > (1 << 24)) return CSRCOLOR_EINVAL;
    if (n == 0) {
        if (ncolors_host) *ncolors_host = 0;
        if (stats) {
            stats->rounds = stats->ncolors = stats->max_degree = 0;
            stats->rows_sorted = 1;
            stats->nnz = 0;
        }
        return CSRCOLOR_OK;
    }
    if (!rowptr || !colors_out) return CSRCOLOR_EINVAL;   // colidx may be NULL when rowptr[n] == 0
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CSRCOLOR_EHIP;
    Workspace* w = get_ws(dev, stream);
    std::lock_guard<std::mutex> lk(w->mu);
    Job J;
    J.n = n;
    J.rowptr = rowptr;
    J.colidx = colidx;
    J.colors_out = colors_out;
    J.opt = parse_opts(opts);
    J.stats = stats;
    int rc = run_job(w, J, nullptr, 0);
    if (rc) return rc;
    if (ncolors_host) *ncolors_host = J.ncolors;
    return CSRCOLOR_OK;
}
}  // namespace

extern "C" {

int csrcolor_color_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* colors_out,
                      int32_t* ncolors_dev, const csrcolor_opts* opts, csrcolor_stats* stats,
                      hipStream_t stream) {
    if (n < 0) return CSRCOLOR_EINVAL;
    if (!opts_valid(opts, true)) return CSRCOLOR_EINVAL;
    if (stats && stats->cap > 0 && stats->cap > (1 << 24)) return CSRCOLOR_EINVAL;
    const int mode = opts ? opts->mode : CSRCOLOR_MODE_AUTO;
    const int algo = opts ? opts->algorithm : CSRCOLOR_ALGO_SGR;
    const bool device = mode == CSRCOLOR_MODE_PERSISTENT ||
                        (mode == CSRCOLOR_MODE_AUTO && !stats && algo == CSRCOLOR_ALGO_SGR);
    if (!device) {
        int32_t nc = 0;
        int rc = color_host(n, rowptr, colidx, colors_out, &nc, opts, stats, stream);
        if (rc) return rc;
        if (ncolors_dev) {
            k_fill<<<1, 64, 0, stream>>>(ncolors_dev, 1, nc);
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) return CSRCOLOR_EHIP;
        }
        return CSRCOLOR_OK;
    }
    if (n == 0) {
        if (stats) {
            stats->rounds = stats->ncolors = stats->max_degree = 0;
            stats->rows_sorted = 1;
            stats->nnz = 0;
        }
        if (ncolors_dev) {
            k_fill<<<1, 64, 0, stream>>>(ncolors_dev, 1, 0);
            if (hipGetLastError() != hipSuccess) return CSRCOLOR_EHIP;
        }
        return CSRCOLOR_OK;
    }
    if (!rowptr || !colors_out) return CSRCOLOR_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CSRCOLOR_EHIP;
    Workspace* w = get_ws(dev, stream);
    std::lock_guard<std::mutex> lk(w->mu);
    Job J;
    J.n = n;
    J.rowptr = rowptr;
    J.colidx = colidx;
    J.colors_out = colors_out;
    J.opt = parse_opts(opts);
    J.opt.mode = CSRCOLOR_MODE_PERSISTENT;
    J.stats = stats;
    return run_device(w, J, nullptr, 0, ncolors_dev, stats != nullptr);
}

int csrcolor_color(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* colors_out,
                   int32_t* ncolors, hipStream_t stream) {
    if (!ncolors) return CSRCOLOR_EINVAL;
    return color_host(n, rowptr, colidx, colors_out, ncolors, nullptr, nullptr, stream);
}

int csrcolor_color_noalloc(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                           int32_t* colors_out, int32_t* ncolors_dev, hipStream_t stream) {
    if (n < 0 || nnz < 0) return CSRCOLOR_EINVAL;
    if ((size_t)n > NA_N || (size_t)nnz > NA_E) return CSRCOLOR_ETOOBIG;
    if (n == 0) {
        if (ncolors_dev) {
            k_fill<<<1, 64, 0, stream>>>(ncolors_dev, 1, 0);
            if (hipGetLastError() != hipSuccess) return CSRCOLOR_EHIP;
        }
        return CSRCOLOR_OK;
    }
    if (!rowptr || !colors_out || (nnz > 0 && !colidx)) return CSRCOLOR_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CSRCOLOR_EHIP;
    if (dev < 0 || dev >= 64) return CSRCOLOR_EINVAL;
    int rc = CSRCOLOR_OK;
    Workspace* w = noalloc_ws(dev, &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    w->stream = stream;
    Job J;
    J.n = n;
    J.rowptr = rowptr;
    J.colidx = colidx;
    J.colors_out = colors_out;
    J.opt.mode = CSRCOLOR_MODE_PERSISTENT;
    J.opt.live = 0;
    J.stats = nullptr;
    J.expect_nnz = nnz;
    KTimer T(w, false);
    return enqueue_device(w, J, nullptr, 0, ncolors_dev, T, true, nullptr);
}

int csrcolor_color_batched(int32_t G, int32_t n_total, const int64_t* voff, const int32_t* rowptr,
                           const int32_t* colidx, int32_t* colors_out, int32_t* ncolors_out,
                           const csrcolor_opts* opts, hipStream_t stream) {
    if (G < 0 || n_total < 0) return CSRCOLOR_EINVAL;
    if (G == 0) return n_total == 0 ? CSRCOLOR_OK : CSRCOLOR_EINVAL;
    if (!voff || !ncolors_out) return CSRCOLOR_EINVAL;
    if (!opts_valid(opts, false)) return CSRCOLOR_EINVAL;
    if (n_total > 0 && (!rowptr || !colors_out)) return CSRCOLOR_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CSRCOLOR_EHIP;
    Workspace* w = get_ws(dev, stream);
    std::lock_guard<std::mutex> lk(w->mu);
    if (n_total > 0) {
        Job J;
        J.n = n_total;
        J.rowptr = rowptr;
        J.colidx = colidx;
        J.colors_out = colors_out;
        J.opt = parse_opts(opts);
        J.stats = nullptr;
        if (J.opt.mode == CSRCOLOR_MODE_PERSISTENT)   // one fused launch, no host wait
            return run_device(w, J, reinterpret_cast<const long long*>(voff), G, ncolors_out, false);
        int rc = run_job(w, J, reinterpret_cast<const long long*>(voff), G);
        if (rc) return rc;
    }
    const int cus = num_cus(dev);
    if (n_total == 0) {
        k_fill<<<(G + WG - 1) / WG, WG, 0, stream>>>(ncolors_out, G, 0);
        if (hipGetLastError() != hipSuccess) return CSRCOLOR_EHIP;
        return hipStreamSynchronize(stream) == hipSuccess ? CSRCOLOR_OK : CSRCOLOR_EHIP;
    }
    k_segmented_max<<<std::min(G, cus * 8), WG, 0, stream>>>(G, reinterpret_cast<const long long*>(voff),
                                                               colors_out, ncolors_out);
    if (hipGetLastError() != hipSuccess) return CSRCOLOR_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return CSRCOLOR_EHIP;
    return CSRCOLOR_OK;
}

int csrcolor_color_multi(int32_t G, const int32_t* n_host, const int64_t* nnz_host,
                         const int32_t* const* rowptr_host, const int32_t* const* colidx_host,
                         int32_t* const* colors_host, int32_t* ncolors_out, const csrcolor_opts* opts,
                         hipStream_t stream) {
    if (G < 0) return CSRCOLOR_EINVAL;
    if (G == 0) return CSRCOLOR_OK;
    if (!n_host || !nnz_host || !rowptr_host || !colidx_host || !colors_host || !ncolors_out)
        return CSRCOLOR_EINVAL;
    if (!opts_valid(opts, false)) return CSRCOLOR_EINVAL;
    long long N = 0, E = 0;
    for (int g = 0; g < G; ++g) {
        if (n_host[g] < 0 || nnz_host[g] < 0) return CSRCOLOR_EINVAL;
        if (!rowptr_host[g] || (n_host[g] > 0 && !colors_host[g]) || (nnz_host[g] > 0 && !colidx_host[g]))
            return CSRCOLOR_EINVAL;
        N += n_host[g];
        E += nnz_host[g];
    }
    if (N >= (1ll << 31) - 1 || E >= (1ll << 31) - 1) return CSRCOLOR_EOVERFLOW;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CSRCOLOR_EHIP;
    Workspace* w = get_ws(dev, stream);
    std::lock_guard<std::mutex> lk(w->mu);
    // size every buffer first: nothing below may reallocate what the union copy filled
    int rc = ensure_capacity(w, (size_t)std::max<long long>(N, 1), 0);
    if (rc) return rc;
    rc = ensure_union(w, (size_t)N, (size_t)E, (size_t)G);
    if (rc) return rc;
    // the staging buffers may still feed an earlier call's copies: wait for the stream
    HIP_TRY(hipStreamSynchronize(stream));
    long long vo = 0, eo = 0;
    int maxn = 0;
    long long maxe = 0;
    for (int g = 0; g < G; ++g) {
        MultiDesc& m = w->u_desc_h[g];
        m.rowptr = rowptr_host[g];
        m.colidx = colidx_host[g];
        m.colors = colors_host[g];
        m.voff = vo;
        m.eoff = eo;
        m.n = n_host[g];
        m.pad = 0;
        m.nnz = nnz_host[g];
        w->u_voff_h[g] = vo;
        vo += n_host[g];
        eo += nnz_host[g];
        maxn = std::max(maxn, n_host[g]);
        maxe = std::max(maxe, (long long)nnz_host[g]);
    }
    w->u_voff_h[G] = vo;
    HIP_TRY(hipMemcpyAsync(w->u_desc, w->u_desc_h, G * sizeof(MultiDesc), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(w->u_voff, w->u_voff_h, (G + 1) * sizeof(long long), hipMemcpyHostToDevice, stream));
    k_init<<<1, WG, 0, stream>>>(w->ctl);
    const long long per = std::max<long long>(maxn, maxe);
    const int gx = (int)std::min<long long>(std::max<long long>((per + WG * 4 - 1) / (WG * 4), 1), 64);
    k_concat<<<dim3(gx, G), WG, 0, stream>>>(w->u_desc, G, w->u_rowptr, w->u_colidx, N, E, w->ctl);
    HIP_TRY(hipGetLastError());
    if ((rc = read_ctl(w))) return rc;
    if (w->ctl_h->err) return CSRCOLOR_EBADCSR;
    if (N > 0) {
        Job J;
        J.n = (int)N;
        J.rowptr = w->u_rowptr;
        J.colidx = E > 0 ? w->u_colidx : nullptr;
        J.colors_out = w->u_colors;
        J.opt = parse_opts(opts);
        J.stats = nullptr;
        rc = run_job(w, J, w->u_voff, G);
        if (rc) return rc;
        const int gxs = (int)std::min<long long>(std::max<long long>((maxn + WG * 4 - 1) / (WG * 4), 1), 64);
        k_scatter<<<dim3(gxs, G), WG, 0, stream>>>(w->u_desc, w->u_colors);
        k_segmented_max<<<std::min(G, num_cus(dev) * 8), WG, 0, stream>>>(G, w->u_voff, w->u_colors, ncolors_out);
    } else {
        k_fill<<<(G + WG - 1) / WG, WG, 0, stream>>>(ncolors_out, G, 0);
    }
    if (hipGetLastError() != hipSuccess) return CSRCOLOR_EHIP;
    return hipStreamSynchronize(stream) == hipSuccess ? CSRCOLOR_OK : CSRCOLOR_EHIP;
}

const char* csrcolor_strerror(int status) {
    switch (status) {
        case CSRCOLOR_OK: return "success";
        case CSRCOLOR_EINVAL: return "invalid argument";
        case CSRCOLOR_EBADCSR: return "malformed CSR (rowptr not monotone from 0, or colidx out of range)";
        case CSRCOLOR_ENOMEM: return "out of memory";
        case CSRCOLOR_EHIP: return "HIP runtime error";
        case CSRCOLOR_EOVERFLOW: return "size exceeds int32 range";
        case CSRCOLOR_ENOTSYM: return "CSR is not symmetric";
        case CSRCOLOR_ELIMIT: return "round limit exceeded";
        case CSRCOLOR_ETIMEOUT: return "a device-wide barrier timed out (the persistent grid was not resident)";
        case CSRCOLOR_ETOOBIG: return "graph larger than the fixed scratch of the allocation-free entry point";
        default: return "unknown status";
    }
}

void csrcolor_release_workspace(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_ws) {
        Workspace* w = kv.second;
        std::lock_guard<std::mutex> l2(w->mu);
        (void)hipSetDevice(w->device);
        (void)hipStreamSynchronize(w->stream);
        free_ws_arrays(w);
        // every handle is reset after it is freed: the next call on this stream starts
        // from an empty workspace and recreates what it needs
        if (w->ctl) (void)hipFree(w->ctl);
        if (w->ubytes) (void)hipFree(w->ubytes);
        if (w->ctl_h) (void)hipHostFree(w->ctl_h);
        if (w->ctl_h2) (void)hipHostFree(w->ctl_h2);
        w->ctl = nullptr;
        w->ubytes = nullptr;
        w->ctl_h = w->ctl_h2 = nullptr;
        for (int i = 0; i < 2; ++i) {
            if (w->pev[i]) (void)hipEventDestroy(w->pev[i]);
            w->pev[i] = nullptr;
        }
        for (hipEvent_t e : w->evs) (void)hipEventDestroy(e);
        w->evs.clear();
        if (w->st_wsize) (void)hipFree(w->st_wsize);
        if (w->st_arcs) (void)hipFree(w->st_arcs);
        w->st_wsize = w->st_arcs = nullptr;
        w->st_cap = 0;
        if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
        w->gexec = nullptr;
        w->gbudget = 0;
        memset(&w->gargs, 0, sizeof(w->gargs));
        if (w->gev) (void)hipEventDestroy(w->gev);
        w->gev = nullptr;
        if (w->gstream) (void)hipStreamDestroy(w->gstream);
        w->gstream = nullptr;
        if (w->plan) (void)hipFree(w->plan);
        w->plan = nullptr;
        if (w->sz_h) (void)hipHostFree(w->sz_h);
        w->sz_h = nullptr;
    }
    (void)hipSetDevice(cur);
}

int64_t csrcolor_workspace_bytes(int32_t G, int64_t n, int64_t nnz) {
    if (G < 0 || n < 0 || nnz < 0) return CSRCOLOR_EINVAL;
    return (int64_t)ws_bound(G, n, nnz);
}

int64_t csrcolor_device_bytes_in_use(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t b = 0;
    for (auto& kv : g_ws) b += ws_bytes_now(kv.second);
    return (int64_t)b;
}

int csrcolor_version(void) { return 100; }

}  // extern "C"
