// Topology-driven variant (Sec. 3.1, Algorithm Topo-GC), kept as an ablation of the
// worklist path: every round is launched over all n vertices with one lane per vertex
// (the paper's baseline mapping); a vertex that is already settled exits at once.  Rows
// longer than TOPO_LONG arcs are handed to the whole wavefront so that one hub does not
// serialise a lane.  The colour word X and the round semantics are those of the worklist
// path (X > 0 settled, X <= 0 uncoloured, FLAG | c tentative), so the colouring is the
// same; only the work per round differs (n vertices visited instead of |W_r|).
#pragma once
#include "sgr_device.h"

namespace csrcolor {

constexpr int TOPO_LONG = 64;   // longer rows are scanned by the whole wavefront
constexpr int TOPO_BMW = 64;    // words of the per-wavefront colour bitmap window (2048 colours)

// Smallest colour >= 1 held by no settled neighbour of row [beg, end), computed by the
// whole wavefront through LDS bitmap windows of 2048 colours (a further window only if
// one is completely forbidden).  Every lane must call with the same row.
__device__ __forceinline__ int topo_wave_mex(const int* __restrict__ colidx, const int* X, int beg, int end,
                                             unsigned* bm) {
    const int lane = __lane_id();
    for (int base = 0;; base += TOPO_BMW * 32) {
        bm[lane] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int e = beg + lane; e < end; e += 64) {
            const int x = X[colidx[e]];
            const int k = x - 1 - base;
            if (x > 0 && (unsigned)k < (unsigned)(TOPO_BMW * 32)) atomicOr(&bm[k >> 5], 1u << (k & 31));
        }
        __builtin_amdgcn_wave_barrier();
        const unsigned wd = bm[lane];
        const unsigned long long z = __ballot(wd != 0xffffffffu);
        __builtin_amdgcn_wave_barrier();
        if (z) {
            const int l = __ffsll((long long)z) - 1;
            const unsigned wl = __shfl(wd, l, 64);
            return base + 32 * l + __ffs(~wl);
        }
    }
}

// FirstFit over V.  Block 0 first books the round: the uncoloured count left by the
// previous round (cnt[par ^ 1][0]) is this round's |W|; a zero means every vertex is
// settled and the launch is a no-op.  It also clears this round's loser counter.
__global__ __launch_bounds__(WG) void k_topo_assign(int n, const int* __restrict__ rowptr,
                                                    const int* __restrict__ colidx, int* X, Ctl* ctl, int par,
                                                    long long* st_wsize, int st_cap) {
    __shared__ unsigned bm[WAVES][TOPO_BMW];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int prev = ctl->cnt[par ^ 1][0];
        if (prev > 0) {
            const int r = ctl->rounds;
            if (st_wsize && r < st_cap) st_wsize[r] = prev;
            ctl->rounds = r + 1;
        }
        ctl->cnt[par][0] = 0;
    }
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const long long stride = (long long)gridDim.x * WG;
    for (long long t = (long long)blockIdx.x * WG + wv * 64; t < n; t += stride) {
        const int v = t + lane < n ? (int)(t + lane) : -1;
        int beg = 0, end = 0;
        bool todo = false;
        if (v >= 0 && X[v] <= 0) {
            beg = rowptr[v];
            end = rowptr[v + 1];
            todo = true;
        }
        const bool longrow = todo && end - beg > TOPO_LONG;
        if (todo && !longrow) {
            // deg <= 64, so the smallest free colour is <= 65
            unsigned long long m = 0;
            for (int e = beg; e < end; ++e) {
                const int x = X[colidx[e]];
                if (x > 0 && x <= 64) m |= 1ull << (x - 1);
            }
            X[v] = FLAG | (~m ? __ffsll((long long)~m) : 65);
        }
        unsigned long long lr = __ballot(longrow);
        while (lr) {
            const int j = __ffsll((long long)lr) - 1;
            lr &= lr - 1;
            const int c = topo_wave_mex(colidx, X, __builtin_amdgcn_readlane(beg, j),
                                        __builtin_amdgcn_readlane(end, j), bm[wv]);
            if (lane == j) X[v] = FLAG | c;
        }
    }
}

// Conflict test over V for the vertices holding a tentative colour: winners settle
// (X = c, out = c - 1), losers keep FLAG | c (uncoloured for the next FirstFit) and are
// counted in cnt[par][0] (one atomic per workgroup).
__global__ __launch_bounds__(WG) void k_topo_detect(int n, const int* __restrict__ rowptr,
                                                    const int* __restrict__ colidx, int* X, int* out, Ctl* ctl,
                                                    int par, int sorted, int rule) {
    __shared__ int red[WAVES];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const long long stride = (long long)gridDim.x * WG;
    int lost_cnt = 0, cmax = 0;
    for (long long t = (long long)blockIdx.x * WG + wv * 64; t < n; t += stride) {
        const int v = t + lane < n ? (int)(t + lane) : -1;
        int beg = 0, end = 0, cv = 0;
        bool todo = false;
        if (v >= 0) {
            const int x = X[v];
            if (x < 0) {
                todo = true;
                cv = x & CMASK;
                beg = rowptr[v];
                end = rowptr[v + 1];
            }
        }
        const bool longrow = todo && end - beg > TOPO_LONG;
        bool lost = false;
        if (todo && !longrow) {
            for (int e = beg; e < end; ++e) {
                const int w = colidx[e];
                if (rule == 0 && sorted && w > v) break;
                if (conflict(rule, rowptr, X, w, v, cv, end - beg)) {
                    lost = true;
                    break;
                }
            }
        }
        unsigned long long lr = __ballot(longrow);
        while (lr) {
            const int j = __ffsll((long long)lr) - 1;
            lr &= lr - 1;
            const int u = __builtin_amdgcn_readlane(v, j);
            const int ub = __builtin_amdgcn_readlane(beg, j);
            const int ue = __builtin_amdgcn_readlane(end, j);
            const int cu = __builtin_amdgcn_readlane(cv, j);
            bool hit = false;
            for (int e0 = ub; e0 < ue; e0 += 64) {
                const int e = e0 + lane;
                bool h = false, stop = false;
                if (e < ue) {
                    const int w = colidx[e];
                    if (rule == 0 && sorted && w > u) stop = true;
                    else h = conflict(rule, rowptr, X, w, u, cu, ue - ub);
                }
                if (__ballot(h)) {
                    hit = true;
                    break;
                }
                if (__ballot(stop)) break;
            }
            if (lane == j) lost = hit;
        }
        if (todo) {
            if (lost) {
                ++lost_cnt;
            } else {
                X[v] = cv;
                out[v] = cv - 1;
                cmax = max(cmax, cv);
            }
        }
    }
    lost_cnt = block_sum(lost_cnt, red);
    cmax = block_max(cmax, red);
    if (threadIdx.x == 0) {
        if (lost_cnt) atomicAdd(&ctl->cnt[par][0], lost_cnt);
        if (cmax) atomicMax(&ctl->maxcolor, cmax);
    }
}

}  // namespace csrcolor
