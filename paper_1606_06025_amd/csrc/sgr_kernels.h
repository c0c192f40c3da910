// Kernels of one speculative-greedy colouring: validation, the round-1 shortcut,
// FirstFit (assign) and conflict test + compaction (detect) per degree bucket.
#pragma once

#include "sgr_device.h"

namespace csrcolor {

// ---------------------------------------------------------------------------
// Control-block reset (a kernel, not a memset, so the sequence can be captured).
// ---------------------------------------------------------------------------
__global__ void k_init(Ctl* ctl) {
    int* p = reinterpret_cast<int*>(ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Structural validation, degree histogram and row-order detection.
// Vertex pass: rowptr[0] == 0, 0 <= rowptr[v] <= rowptr[v+1] <= rowptr[n];
// counts descents colidx[e] < colidx[e-1] at positions e that start a row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_validate_rows(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ colidx, Ctl* ctl,
                                                      int twave) {
    const int nnz = rowptr[n];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->nnz = nnz;
    int mydeg = 0;
    int hist[NB] = {0, 0, 0, 0, 0};
    int bad = 0, desc = 0;
    for (long long v = (long long)blockIdx.x * WG + threadIdx.x; v < n; v += (long long)gridDim.x * WG) {
        const int beg = rowptr[v], end = rowptr[v + 1];
        const bool ok = beg >= 0 && beg <= end && end <= nnz && (v != 0 || beg == 0);
        if (!ok) { bad = 1; continue; }
        const int deg = end - beg;
        mydeg = max(mydeg, deg);
        if (deg > 0) {
            const int bk = bucket_of(deg, twave);
#pragma unroll
            for (int b = 0; b < NB; ++b) hist[b] += (bk == b);
            if (beg > 0 && colidx[beg] < colidx[beg - 1]) desc++;
        }
    }
    if (nnz < 0 || (colidx == nullptr && nnz != 0)) bad = 1;
    mydeg = wave_max(mydeg);
    unsigned long long anybad = __ballot(bad);
    int d = desc;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off, 64);
    int h[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int x = hist[b];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        h[b] = x;
    }
    if (__lane_id() == 0) {
        if (anybad) atomicOr(&ctl->err, 1);
        if (mydeg) atomicMax(&ctl->maxdeg, mydeg);
        if (d) atomicAdd(&ctl->desc_bound, d);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (h[b]) atomicAdd(&ctl->hist[b], h[b]);
    }
}

// Arc pass: colidx in [0, n); counts all descents.  Launched only after the vertex
// pass found rowptr consistent, so [0, rowptr[n]) is the caller's colidx extent.
__global__ __launch_bounds__(WG) void k_validate_arcs(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ colidx, Ctl* ctl) {
    const long long nnz = rowptr[n];
    int bad = 0, desc = 0;
    for (long long e = (long long)blockIdx.x * WG + threadIdx.x; e < nnz; e += (long long)gridDim.x * WG) {
        const int w = colidx[e];
        if ((unsigned)w >= (unsigned)n) bad = 1;
        if (e > 0 && w < colidx[e - 1]) desc++;
    }
    unsigned long long anybad = __ballot(bad);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) desc += __shfl_xor(desc, off, 64);
    if (__lane_id() == 0) {
        if (anybad) atomicOr(&ctl->err, 2);
        if (desc) atomicAdd(&ctl->desc_total, desc);
    }
}

// Symmetry check (sorted rows): arc (v, w) needs v in row w.  One thread per vertex
// row entry; binary search in row w.
__global__ __launch_bounds__(WG) void k_check_symmetric(int n, const int* __restrict__ rowptr,
                                                        const int* __restrict__ colidx, Ctl* ctl) {
    int bad = 0;
    for (long long v = (long long)blockIdx.x * WG + threadIdx.x; v < n; v += (long long)gridDim.x * WG) {
        for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            const int w = colidx[e];
            int lo = rowptr[w], hi = rowptr[w + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (colidx[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= rowptr[w + 1] || colidx[lo] != v) bad = 1;
        }
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&ctl->err, 4);
}

// ---------------------------------------------------------------------------
// Round 1 shortcut.  With an all-zero snapshot FirstFit gives colour 1 to every
// vertex, so v is requeued iff it has a neighbour w < v.  For sorted rows that is
// one test of the row's first entry.  Winners are final with colour 1; losers are
// pushed to the worklist of their degree bucket.
// One workgroup handles 4*WG consecutive vertices and compacts them per bucket in
// LDS, so there are at most NB global atomics per workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_round1(int n, const int* __restrict__ rowptr,
                                               const int* __restrict__ colidx, int* X, int* out,
                                               int* wl1, Ctl* ctl, int sorted, int twave,
                                               Seg seg) {
    constexpr int ITER = 4;
    __shared__ int buf[WAVES][NB][ITER * 64];
    __shared__ int wcnt[WAVES][NB];
    __shared__ int wbase[WAVES][NB];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int cnt[NB] = {0, 0, 0, 0, 0};
    const long long chunk0 = (long long)blockIdx.x * (ITER * WG);
    for (int it = 0; it < ITER; ++it) {
        const long long vv = chunk0 + it * WG + threadIdx.x;
        bool lose = false;
        int bkt = -1;
        if (vv < n) {
            const int v = (int)vv;
            const int beg = rowptr[v], end = rowptr[v + 1];
            if (end > beg) {
                if (sorted) {
                    lose = colidx[beg] < v;
                } else {
                    for (int e = beg; e < end; ++e)
                        if (colidx[e] < v) { lose = true; break; }
                }
            }
            if (lose) {
                X[v] = FLAG | 1;
                bkt = bucket_of(end - beg, twave);
            } else {
                X[v] = 1;
                out[v] = 0;
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const unsigned long long m = __ballot(bkt == b);
            if (bkt == b) buf[wv][b][cnt[b] + __popcll(m & lanemask_lt())] = (int)vv;
            cnt[b] += __popcll(m);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) wcnt[wv][b] = cnt[b];
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        const int b = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += wcnt[w][b];
        int base = tot ? atomicAdd(&ctl->cnt[1][b], tot) : 0;
        for (int w = 0; w < WAVES; ++w) { wbase[w][b] = base; base += wcnt[w][b]; }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int* dst = wl1 + seg.s[b] + wbase[wv][b];
        for (int k = lane; k < cnt[b]; k += 64) dst[k] = buf[wv][b][k];
    }
}

// ---------------------------------------------------------------------------
// Shared LDS layout of the round kernels.
// ---------------------------------------------------------------------------
struct RoundLds {
    union {
        int lbuf[WAVES * WAVE_CAP];   // detect: per-wavefront loser buffers
        unsigned ovf[WAVES * OVW];    // assign, wave bucket: overflow colour bitmaps
        unsigned bm[BMW];             // assign, workgroup bucket: colour window bitmap
    };
    int wcnt[WAVES];
    int wbase[WAVES];
    int red[WAVES];
    long long red64[WAVES];
    int sh;
    int flag;
};

__device__ __forceinline__ void locate_block(const RoundArgs& a, int& b, int& j, int& nbk) {
    const int bid = blockIdx.x;
    b = 0;
#pragma unroll
    for (int k = 1; k < NB; ++k)
        if (bid >= a.boff[k]) b = k;
    nbk = a.boff[b + 1] - a.boff[b];
    j = bid - a.boff[b];
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous
    // slice of the bucket's worklist so neighbouring vertices share an L2.
    if ((nbk & 7) == 0 && (a.boff[b] & 7) == 0) {
        const int per = nbk >> 3;
        j = (j & 7) * per + (j >> 3);
    }
}

// ---------------------------------------------------------------------------
// FirstFit (Sec. 3, FirstFit routine, with the bitset of Sec. 3.2): colour =
// smallest c > 0 with bit c-1 clear in the OR of the neighbours' settled colours.
// ---------------------------------------------------------------------------

// G lanes per vertex, degree <= G <= 32, so the mex is <= 33 and one 64-bit mask
// in registers holds every colour that can matter.
template <int G>
__device__ __forceinline__ void assign_groups(const RoundArgs& a, const int* list, int lo, int hi,
                                              long long& arcs) {
    constexpr int GPW = WG / G;
    const int gl = threadIdx.x & (G - 1);
    const int gid = threadIdx.x / G;
    for (int base = lo; base < hi; base += GPW) {
        const int i = base + gid;
        const bool act = i < hi;
        int v = 0, beg = 0, end = 0;
        if (act) {
            v = list[i];
            beg = a.rowptr[v];
            end = a.rowptr[v + 1];
        }
        unsigned long long m = 0;
        for (int e = beg + gl; e < end; e += G) {
            const int x = a.X[a.colidx[e]];
            if (x > 0 && x <= 64) m |= 1ull << (x - 1);
        }
        m = group_or<G>(m);
        if (act && gl == 0) {
            a.X[v] = FLAG | __ffsll((long long)~m);
            arcs += end - beg;
        }
    }
}

// One wavefront per vertex (32 < degree <= t_wave <= 1024): colours 1..64 in a
// register mask, colours 65..1088 in a per-wavefront LDS bitmap.
__device__ __forceinline__ void assign_waves(const RoundArgs& a, const int* list, int lo, int hi,
                                             unsigned* ovf, long long& arcs) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    unsigned* my = ovf + wv * OVW;
    for (int i = lo + wv; i < hi; i += WAVES) {
        const int v = list[i];
        const int beg = a.rowptr[v], end = a.rowptr[v + 1];
        if (lane < OVW) my[lane] = 0;
        __builtin_amdgcn_wave_barrier();
        unsigned long long m = 0;
        for (int e = beg + lane; e < end; e += 64) {
            const int x = a.X[a.colidx[e]];
            if (x > 0) {
                if (x <= 64) {
                    m |= 1ull << (x - 1);
                } else {
                    const int k = x - 65;
                    if (k < OVW * 32) atomicOr(&my[k >> 5], 1u << (k & 31));
                }
            }
        }
        m = group_or<64>(m);
        __builtin_amdgcn_wave_barrier();
        int c;
        if (~m) {
            c = __ffsll((long long)~m);
        } else {
            const unsigned word = lane < OVW ? my[lane] : 0xffffffffu;
            const unsigned long long z = __ballot(word != 0xffffffffu);
            if (z == 0) {
                if (lane == 0) atomicOr(&a.ctl->err, 8);
                c = 1;
            } else {
                const int l = __ffsll((long long)z) - 1;
                const unsigned wl = __shfl(word, l, 64);
                c = 65 + 32 * l + __ffs(~wl) - 1;
            }
        }
        if (lane == 0) {
            a.X[v] = FLAG | c;
            arcs += end - beg;
        }
    }
}

// One workgroup per vertex (degree > t_wave): LDS bitmap over a window of 32768
// colours; a further window is scanned only if every colour of one is forbidden.
__device__ __forceinline__ void assign_wg(const RoundArgs& a, const int* list, int cnt, RoundLds& s,
                                          long long& arcs) {
    for (;;) {
        if (threadIdx.x == 0) s.sh = atomicAdd(&a.ctl->dyn[0][4], 1);
        __syncthreads();
        const int i = s.sh;
        __syncthreads();
        if (i >= cnt) break;
        const int v = list[i];
        const int beg = a.rowptr[v], end = a.rowptr[v + 1];
        int base = 0, c = 0;
        for (;;) {
            for (int k = threadIdx.x; k < BMW; k += WG) s.bm[k] = 0;
            __syncthreads();
            for (int e = beg + threadIdx.x; e < end; e += WG) {
                const int x = a.X[a.colidx[e]];
                const int k = x - 1 - base;
                if (x > 0 && (unsigned)k < (unsigned)(BMW * 32)) atomicOr(&s.bm[k >> 5], 1u << (k & 31));
            }
            __syncthreads();
            int best = 0x7fffffff;
            for (int k = threadIdx.x; k < BMW; k += WG) {
                const unsigned wd = s.bm[k];
                if (wd != 0xffffffffu) best = min(best, k * 32 + __ffs(~wd) - 1);
            }
            best = block_min(best, s.red);
            if (best != 0x7fffffff) { c = base + best + 1; break; }
            base += BMW * 32;
        }
        if (threadIdx.x == 0) {
            a.X[v] = FLAG | c;
            arcs += end - beg;
        }
    }
}

__global__ __launch_bounds__(WG) void k_assign(RoundArgs a) {
    __shared__ RoundLds s;
    int b, j, nbk;
    locate_block(a, b, j, nbk);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NB; ++k) {
            a.ctl->cnt[a.par_out][k] = 0;
            a.ctl->dyn[1][k] = 0;
        }
    }
    const int cnt = a.ctl->cnt[a.par_in][b];
    const int* list = a.wl_in + a.seg[b];
    const int lo = (int)((long long)j * cnt / nbk);
    const int hi = (int)((long long)(j + 1) * cnt / nbk);
    long long arcs = 0;
    switch (b) {
        case 0: assign_groups<8>(a, list, lo, hi, arcs); break;
        case 1: assign_groups<16>(a, list, lo, hi, arcs); break;
        case 2: assign_groups<32>(a, list, lo, hi, arcs); break;
        case 3: assign_waves(a, list, lo, hi, s.ovf, arcs); break;
        default: assign_wg(a, list, cnt, s, arcs); break;
    }
    if (a.st_arcs && a.round < a.st_cap) {
        const long long t = block_sum64(arcs, s.red64);
        if (threadIdx.x == 0 && t) atomicAdd((unsigned long long*)&a.st_arcs[a.round], (unsigned long long)t);
    }
}

// ---------------------------------------------------------------------------
// Conflict test (Sec. 3, ConflictResolve, with the requeue direction fixed to the
// higher id) + colour clearing + worklist push by in-LDS prefix (Sec. 3.1).
// A vertex loses iff some neighbour w < v holds the same tentative colour.  With
// sorted rows the scan of a row stops at the first w >= v.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void settle(const RoundArgs& a, int v, int cv, int& cmax) {
    a.X[v] = cv;
    a.out[v] = cv - 1;
    cmax = max(cmax, cv);
}

// Writes the per-wavefront loser buffers to the global worklist with one atomic
// per workgroup.  `wc` is the calling wavefront's count (uniform).
__device__ __forceinline__ void flush_losers(RoundLds& s, int wc, int* outl, int* cnt_out) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    if (lane == 0) s.wcnt[wv] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += s.wcnt[w];
        int base = tot ? atomicAdd(cnt_out, tot) : 0;
        for (int w = 0; w < WAVES; ++w) { s.wbase[w] = base; base += s.wcnt[w]; }
    }
    __syncthreads();
    const int* src = s.lbuf + wv * WAVE_CAP;
    int* dst = outl + s.wbase[wv];
    for (int k = lane; k < wc; k += 64) dst[k] = src[k];
    __syncthreads();
}

template <int G>
__device__ __forceinline__ void detect_groups(const RoundArgs& a, const int* list, int lo, int hi,
                                              RoundLds& s, int* outl, int* cnt_out, int& cmax) {
    constexpr int GPW = WG / G;
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int gl = threadIdx.x & (G - 1);
    const int gid = threadIdx.x / G;
    const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const int gshift = lane & ~(G - 1);
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wc = 0;
        for (int base = s0; base < s1; base += GPW) {
            const int i = base + gid;
            const bool act = i < s1;
            bool lost = false;
            int v = 0;
            if (act) {
                v = list[i];
                const int beg = a.rowptr[v], end = a.rowptr[v + 1];
                const int cv = a.X[v] & CMASK;
                for (int e0 = beg; e0 < end; e0 += G) {
                    const int e = e0 + gl;
                    const int w = e < end ? a.colidx[e] : 0x7fffffff;
                    const bool hit = w < v && (a.X[w] & CMASK) == cv;
                    const bool stop = a.sorted && w >= v;
                    const unsigned long long bh = (__ballot(hit) >> gshift) & gmask;
                    const unsigned long long bs = (__ballot(stop) >> gshift) & gmask;
                    if (bh) { lost = true; break; }
                    if (bs) break;
                }
                if (!lost && gl == 0) settle(a, v, cv, cmax);
            }
            const unsigned long long lm = __ballot(act && gl == 0 && lost);
            if (act && gl == 0 && lost) mybuf[wc + __popcll(lm & lanemask_lt())] = v;
            wc += __popcll(lm);
        }
        flush_losers(s, wc, outl, cnt_out);
    }
}

__device__ __forceinline__ void detect_waves(const RoundArgs& a, const int* list, int lo, int hi,
                                             RoundLds& s, int* outl, int* cnt_out, int& cmax) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wc = 0;
        for (int i = s0 + wv; i < s1; i += WAVES) {
            const int v = list[i];
            const int beg = a.rowptr[v], end = a.rowptr[v + 1];
            const int cv = a.X[v] & CMASK;
            bool lost = false;
            for (int e0 = beg; e0 < end; e0 += 64) {
                const int e = e0 + lane;
                const int w = e < end ? a.colidx[e] : 0x7fffffff;
                const bool hit = w < v && (a.X[w] & CMASK) == cv;
                const bool stop = a.sorted && w >= v;
                if (__ballot(hit)) { lost = true; break; }
                if (__ballot(stop)) break;
            }
            if (lost) {
                if (lane == 0) mybuf[wc] = v;
                ++wc;
            } else if (lane == 0) {
                settle(a, v, cv, cmax);
            }
        }
        flush_losers(s, wc, outl, cnt_out);
    }
}

__device__ __forceinline__ void detect_wg(const RoundArgs& a, const int* list, int cnt, RoundLds& s,
                                          int* outl, int* cnt_out, int& cmax) {
    for (;;) {
        if (threadIdx.x == 0) s.sh = atomicAdd(&a.ctl->dyn[1][4], 1);
        __syncthreads();
        const int i = s.sh;
        __syncthreads();
        if (i >= cnt) break;
        const int v = list[i];
        const int beg = a.rowptr[v], end = a.rowptr[v + 1];
        const int cv = a.X[v] & CMASK;
        bool lost = false;
        for (int e0 = beg; e0 < end; e0 += WG) {
            const int e = e0 + threadIdx.x;
            const int w = e < end ? a.colidx[e] : 0x7fffffff;
            const bool hit = w < v && (a.X[w] & CMASK) == cv;
            const bool stop = a.sorted && w >= v;
            const int anyhit = __syncthreads_or(hit);
            const int anystop = __syncthreads_or(stop);
            if (anyhit) { lost = true; break; }
            if (anystop) break;
        }
        if (threadIdx.x == 0) {
            if (lost) {
                const int p = atomicAdd(cnt_out, 1);
                outl[p] = v;
            } else {
                settle(a, v, cv, cmax);
            }
        }
    }
}

__global__ __launch_bounds__(WG) void k_detect(RoundArgs a) {
    __shared__ RoundLds s;
    int b, j, nbk;
    locate_block(a, b, j, nbk);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < NB; ++k) {
            tot += a.ctl->cnt[a.par_in][k];
            a.ctl->dyn[0][k] = 0;
        }
        if (tot > 0) {
            a.ctl->rounds = a.round + 1;
            if (a.st_wsize && a.round < a.st_cap) a.st_wsize[a.round] = tot;
        }
    }
    const int cnt = a.ctl->cnt[a.par_in][b];
    const int* list = a.wl_in + a.seg[b];
    int* outl = a.wl_out + a.seg[b];
    int* cnt_out = &a.ctl->cnt[a.par_out][b];
    const int lo = (int)((long long)j * cnt / nbk);
    const int hi = (int)((long long)(j + 1) * cnt / nbk);
    int cmax = 0;
    switch (b) {
        case 0: detect_groups<8>(a, list, lo, hi, s, outl, cnt_out, cmax); break;
        case 1: detect_groups<16>(a, list, lo, hi, s, outl, cnt_out, cmax); break;
        case 2: detect_groups<32>(a, list, lo, hi, s, outl, cnt_out, cmax); break;
        case 3: detect_waves(a, list, lo, hi, s, outl, cnt_out, cmax); break;
        default: detect_wg(a, list, cnt, s, outl, cnt_out, cmax); break;
    }
    cmax = block_max(cmax, s.red);
    if (threadIdx.x == 0 && cmax > 0) atomicMax(&a.ctl->maxcolor, cmax);
}

// Per-graph colour count of a batched run: ncolors[g] = 1 + max colour in graph g.
__global__ __launch_bounds__(WG) void k_segmented_max(int G, const long long* __restrict__ voff,
                                                      const int* __restrict__ colors, int* ncolors) {
    __shared__ int red[WAVES];
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const long long v0 = voff[g], v1 = voff[g + 1];
        int m = -1;
        for (long long v = v0 + threadIdx.x; v < v1; v += WG) m = max(m, colors[v]);
        m = block_max(m, red);
        if (threadIdx.x == 0) ncolors[g] = m + 1;
    }
}

__global__ void k_fill(int* p, int count, int value) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = value;
}

// Batched validation: voff[0] == 0, non-decreasing, voff[G] == n_total, and every
// arc of graph g stays inside graph g.
__global__ __launch_bounds__(WG) void k_validate_batch(int G, int n_total, const long long* __restrict__ voff,
                                                       const int* __restrict__ rowptr,
                                                       const int* __restrict__ colidx, Ctl* ctl) {
    int bad = 0;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const long long v0 = voff[g], v1 = voff[g + 1];
        if ((g == 0 && v0 != 0) || v0 < 0 || v0 > n_total || v1 < v0 || v1 > n_total ||
            (g == G - 1 && v1 != n_total)) {
            bad = 1;
            continue;
        }
        const long long e0 = rowptr[v0], e1 = rowptr[v1];
        for (long long e = e0 + threadIdx.x; e < e1; e += WG) {
            const int w = colidx[e];
            if (w < v0 || w >= v1) bad = 1;
        }
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&ctl->err, 16);
}

}  // namespace csrcolor
