// Kernels of one speculative-greedy colouring: validation, the round-1 shortcut and
// the conflict-test launches (worklists per degree bucket; flag scans with wake flags).
#pragma once

#include "sgr_device.h"
#include "sgr_round.h"
#include "sgr_wake.h"

namespace csrcolor {

// ---------------------------------------------------------------------------
// Control-block reset (a kernel, not a memset, so the sequence can be captured).
// ---------------------------------------------------------------------------
__global__ void k_init(Ctl* ctl) {
    int* p = reinterpret_cast<int*>(ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Structural validation, degree histogram and row-order detection, two launches.
// Vertex pass: rowptr[0] == 0, 0 <= rowptr[v] <= rowptr[v+1] <= rowptr[n], and
// rowptr[n] equal to the caller's arc count when one is given (expect_nnz >= 0; on a
// mismatch no colidx entry is read); degree histogram, largest degree, arcs of the
// rows longer than WAKE_DEG; counts descents colidx[e] < colidx[e-1] at positions e
// that start a non-empty row.
// Arc pass, only once the vertex pass found rowptr consistent (so [0, rowptr[n]) is
// the caller's colidx extent): colidx[e] in [0, n); counts all descents.  Rows are
// sorted iff both descent counts agree.
// ---------------------------------------------------------------------------
constexpr int VROWS = 4;   // vertices per thread and loop pass of the vertex pass
constexpr int VQUADS = 4;  // 16-byte quads of colidx per lane and loop pass of the arc pass

__global__ __launch_bounds__(WG) void k_validate_rows(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ colidx, Ctl* ctl, int twave,
                                                      int tsplit, long long expect_nnz, int tiles) {
    const int nnz = rowptr[n];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->nnz = nnz;
    const bool stated = expect_nnz < 0 || (long long)nnz == expect_nnz;
    int mydeg = 0;
    int hist[NB] = {};
    int bad = 0, desc = 0, chunks = 0;
    long long big = 0;
    const long long stride = (long long)gridDim.x * WG * VROWS;
    for (long long v0 = (long long)blockIdx.x * WG * VROWS + threadIdx.x; v0 < n; v0 += stride) {
        int beg[VROWS], end[VROWS], c0[VROWS], c1[VROWS];
        bool ok[VROWS];
#pragma unroll
        for (int k = 0; k < VROWS; ++k) {
            const long long v = v0 + (long long)k * WG;
            beg[k] = 0;
            end[k] = 0;
            if (v < n) {
                beg[k] = rowptr[v];
                end[k] = rowptr[v + 1];
            }
            ok[k] = stated && beg[k] >= 0 && beg[k] <= end[k] && end[k] <= nnz && (v != 0 || beg[k] == 0);
        }
#pragma unroll
        for (int k = 0; k < VROWS; ++k) {
            c0[k] = 0;
            c1[k] = 0;
            // a non-empty valid row: colidx[beg] and colidx[beg - 1] lie in [0, nnz)
            if (ok[k] && end[k] > beg[k] && beg[k] > 0) {
                c0[k] = colidx[beg[k]];
                c1[k] = colidx[beg[k] - 1];
            }
        }
#pragma unroll
        for (int k = 0; k < VROWS; ++k) {
            if (v0 + (long long)k * WG >= n) continue;
            if (!ok[k]) { bad = 1; continue; }
            const int deg = end[k] - beg[k];
            mydeg = max(mydeg, deg);
            if (deg > WAKE_DEG) big += deg;
            if (deg > 0) {
                const int bk = bucket_of(deg, tiles, twave, tsplit);
                if (bk == BSPLIT) chunks += split_chunks(deg);
#pragma unroll
                for (int b = 0; b < NB; ++b) hist[b] += (bk == b);
                if (c0[k] < c1[k]) desc++;
            }
        }
    }
    if (nnz < 0 || !stated || (colidx == nullptr && nnz != 0)) bad = 1;
    __shared__ int red[WAVES];
    bad = block_max(bad, red);
    mydeg = block_max(mydeg, red);
    desc = block_sum(desc, red);
    chunks = block_sum(chunks, red);
    __shared__ long long red64[WAVES];
    big = block_sum64(big, red64);
#pragma unroll
    for (int b = 0; b < NB; ++b) hist[b] = block_sum(hist[b], red);
    if (threadIdx.x == 0) {
        if (bad) atomicOr(&ctl->err, ERR_ROWPTR);
        if (chunks) atomicAdd(&ctl->hchunks, chunks);
        if (big) atomicAdd((unsigned long long*)&ctl->bigarcs, (unsigned long long)big);
        if (mydeg) atomicMax(&ctl->maxdeg, mydeg);
        if (desc) atomicAdd(&ctl->desc_bound, desc);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (hist[b]) atomicAdd(&ctl->hist[b], hist[b]);
    }
}

// Arc pass: the wavefronts stream colidx as aligned 16-byte quads (quad q holds the
// positions 4q - mis .. 4q - mis + 3, mis = the array's offset in ints from a 16-byte
// boundary; positions outside [0, nnz) are ignored, and they share their quad's 16
// bytes with a valid position).  The position before a quad's first one is the last
// one of the previous lane's quad, or read once per wavefront.
__global__ __launch_bounds__(WG) void k_validate_arcs(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ colidx, Ctl* ctl) {
    if (ctl->err) return;   // rowptr already failed: [0, rowptr[n]) is not trustworthy
    const long long nnz = rowptr[n];
    const int blk = (int)blockIdx.x, nblk = (int)gridDim.x;
    int bad = 0, desc = 0;
    if (nnz > 0) {
        const int lane = __lane_id();
        const int mis = (int)((reinterpret_cast<uintptr_t>(colidx) >> 2) & 3);
        const int4* base = reinterpret_cast<const int4*>(colidx - mis);
        const long long nq = (nnz + mis + 3) >> 2;
        const long long step = (long long)nblk * WAVES * 64 * VQUADS;
        for (long long q0 = ((long long)blk * WAVES + (threadIdx.x >> 6)) * 64 * VQUADS; q0 < nq; q0 += step) {
            int4 val[VQUADS];
#pragma unroll
            for (int u = 0; u < VQUADS; ++u) {
                const long long q = q0 + 64 * u + lane;
                val[u] = q < nq ? base[q] : make_int4(0, 0, 0, 0);
            }
            const long long e00 = 4 * q0 - mis;   // position of the wavefront's first element
            const int before = e00 > 0 ? colidx[e00 - 1] : 0;
#pragma unroll
            for (int u = 0; u < VQUADS; ++u) {
                const long long q = q0 + 64 * u + lane;
                int prev = __shfl_up(val[u].w, 1, 64);
                const int last_prev_u = u > 0 ? __shfl(val[u > 0 ? u - 1 : 0].w, 63, 64) : before;
                if (lane == 0) prev = last_prev_u;
                const int x[4] = {val[u].x, val[u].y, val[u].z, val[u].w};
                const long long e0 = 4 * q - mis;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const long long e = e0 + k;
                    if (q < nq && e >= 0 && e < nnz) {
                        if ((unsigned)x[k] >= (unsigned)n) bad = 1;
                        const int pv = k == 0 ? prev : x[k - 1];
                        if (e > 0 && x[k] < pv) desc++;
                    }
                }
            }
        }
    }
    __shared__ int red[WAVES];
    bad = block_max(bad, red);
    desc = block_sum(desc, red);
    if (threadIdx.x == 0) {
        if (bad) atomicOr(&ctl->err, ERR_COLIDX);
        if (desc) atomicAdd(&ctl->desc_total, desc);
    }
}

// Symmetry check (sorted rows): arc (v, w) needs v in row w.  One thread per vertex
// row entry; binary search in row w.  It runs only on a graph the structural passes
// accepted (every row bound and id in range) and whose rows are sorted (the search
// needs them sorted): otherwise it returns, flagging unsorted rows.
__global__ __launch_bounds__(WG) void k_check_symmetric(int n, const int* __restrict__ rowptr,
                                                        const int* __restrict__ colidx, Ctl* ctl) {
    if (ctl->err) return;
    if (ctl->desc_total != ctl->desc_bound) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->err, ERR_UNSORTED);
        return;
    }
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
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&ctl->err, ERR_ASYM);
}

// ---------------------------------------------------------------------------
// Round 1 shortcut.  With an all-zero snapshot FirstFit gives colour 1 to every
// vertex, so v is requeued iff it has a neighbour that beats it: under the id rule
// a neighbour w < v, which for sorted rows is one test of the row's first entry.
// Otherwise the row is scanned up to its first beater: by one lane for rows of at
// most R1_LANE arcs, by the wavefront for rows of at most R1_WAVE arcs and by the
// whole workgroup beyond (a winning hub reads its whole row).  Winners are final
// with colour 1; losers are pushed to the worklist of their degree bucket.
// One workgroup handles 4*WG consecutive vertices and compacts them per bucket in
// LDS, so there are at most NB global atomics per workgroup.
// ---------------------------------------------------------------------------
constexpr int R1_LANE = 64;
constexpr int R1_WAVE = 4096;
constexpr int R1_NONE = 0x7fffffff;

// First entry of row [beg, end) of v that beats v, scanned by one lane, four entries
// in flight; -1 if none.
__device__ __forceinline__ int first_beater_lane(int rule, const int* __restrict__ rowptr,
                                                 const int* __restrict__ colidx, int v, int beg, int end) {
    const int dv = end - beg;
    for (long long e = beg; e < end; e += 4) {   // (64-bit: end may lie near the int range's top)
        int w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = e + k < end ? colidx[e + k] : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (w[k] >= 0 && w[k] != v && beats(rule, rowptr, w[k], v, dv)) return w[k];
    }
    return -1;
}

// The same scanned by the wavefront, 256 entries a step (entry beg + 64k + lane in
// step slot k); every lane returns the first beater in row order, or -1.
__device__ __forceinline__ int first_beater_wave(int rule, const int* __restrict__ rowptr,
                                                 const int* __restrict__ colidx, int v, int beg, int end) {
    const int lane = __lane_id();
    const int dv = end - beg;
    for (long long base = beg; base < end; base += 4 * 64) {
        int w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long long e = base + k * 64 + lane;
            w[k] = e < end ? colidx[e] : -1;
        }
        bool b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = w[k] >= 0 && w[k] != v && beats(rule, rowptr, w[k], v, dv);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned long long m = __ballot(b[k]);
            if (m) return __shfl(w[k], __ffsll((long long)m) - 1);
        }
    }
    return -1;
}
__device__ __forceinline__ void round1_body(int n, const int* __restrict__ rowptr,
                                            const int* __restrict__ colidx, int* X, int* out,
                                            int* wl1, Ctl* ctl, int sorted, int twave, int tsplit,
                                            const int* seg, int* cstart1, int* owner1, unsigned* F, int nnz,
                                            int rule, int jp, int* hint, int* llen, int* clen,
                                            unsigned long long* lb1, int fbytes, unsigned char* dirty,
                                            unsigned char* rflag, unsigned char* aflag, int* srnd,
                                            unsigned long long* Fs, unsigned char* Fq, int4* crec1, int tiles) {
    constexpr int ITER = 4;
    __shared__ int buf[WAVES][NB][ITER * 64];
    __shared__ int wcnt[WAVES][NB];
    __shared__ int wbase[WAVES][NB];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int cnt[NB] = {};
    // wake flags (rflag): a loser of at most WAKE_DEG arcs is not listed but sleeps, or
    // keeps its test flag when its hint is longer; every neighbour of a winner (a loser
    // holding colour 1) gets its recolour flag; winners record their settling round
    PushCtx P;
    P.F = F;
    P.rowptr = rowptr;
    P.colidx = colidx;
    P.nnz = nnz;
    P.bytes = fbytes != 0;
    P.dirty = dirty;
    P.Fq = rflag ? nullptr : Fq;
    P.X = X;
    P.rflag = rflag;
    P.Fs = Fs;
    P.all_tentative = true;
    P.nbytes = nullptr;
    P.loaded = false;
    // SGR: this is round 1.  JP: this only builds W_1 (every vertex with a neighbour;
    // an isolated vertex is alone in its neighbourhood and takes colour 1 here), and
    // the conflict-test launches count the rounds.
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->rounds = jp ? 0 : 1;
    // ordered mode (lb1): the block works on the vertex range of its ticket, and each
    // bucket's run is placed after the runs of the lower tickets (look-back), so every
    // worklist segment starts in ascending id order
    __shared__ int ticket;
    // rows scanned by the whole workgroup: owners (thread, vertex, row bounds) per pass,
    // and three rotating slots for the first beater's row position of each step
    __shared__ int r1cnt[ITER];
    __shared__ int r1own[WG][4];
    __shared__ int r1pos[3];
    if (threadIdx.x == 0) {
        ticket = lb1 ? atomicAdd(&ctl->tk1, 1) : (int)blockIdx.x;
        for (int i = 0; i < ITER; ++i) r1cnt[i] = 0;
        for (int i = 0; i < 3; ++i) r1pos[i] = R1_NONE;
    }
    __syncthreads();
    const bool scan_rows = !jp && !(rule == 0 && sorted);
    int slot = 0;
    const int unit = ticket;
    const long long chunk0 = (long long)unit * (ITER * WG);
    for (int it = 0; it < ITER; ++it) {
        // wavefront wv owns the 64*ITER consecutive vertices starting at chunk0 + wv*64*ITER,
        // so concatenating the per-wavefront buffers keeps ascending vertex order
        const long long vv = chunk0 + (long long)wv * (64 * ITER) + it * 64 + lane;
        bool lose = false;
        bool winpush = false;   // push mode: a round-1 winner with neighbours
        int bkt = -1;
        int wbeg = 0, wend = 0;
        int beg = 0, end = 0;
        int by = -1;   // the neighbour that beat v (conflict hint for the next rounds)
        bool pend = false;
        if (vv < n) {
            const int v = (int)vv;
            beg = rowptr[v];
            end = rowptr[v + 1];
            if (jp) {
                lose = end > beg;
            } else if (end > beg) {
                if (!scan_rows) {
                    by = colidx[beg];
                    lose = by < v;
                } else if (end - beg <= R1_LANE) {
                    // all tentative colours are 1: requeued iff some neighbour beats v
                    by = first_beater_lane(rule, rowptr, colidx, v, beg, end);
                    lose = by >= 0;
                } else {
                    pend = true;
                }
            }
        }
        if (scan_rows) {
            // longer rows: the wavefront scans each in turn, the longest the workgroup
            unsigned long long pm = __ballot(pend && end - beg <= R1_WAVE);
            while (pm) {
                const int L = __ffsll((long long)pm) - 1;
                pm &= pm - 1;
                const int w = first_beater_wave(rule, rowptr, colidx, __shfl((int)vv, L), __shfl(beg, L),
                                                __shfl(end, L));
                if (lane == L) {
                    by = w;
                    lose = w >= 0;
                    pend = false;
                }
            }
            if (pend) {
                const int s = atomicAdd(&r1cnt[it], 1);
                r1own[s][0] = threadIdx.x;
                r1own[s][1] = (int)vv;
                r1own[s][2] = beg;
                r1own[s][3] = end;
            }
            __syncthreads();
            const int nbig = r1cnt[it];
            for (int j = 0; j < nbig; ++j) {
                const int own = r1own[j][0], rv = r1own[j][1], rb = r1own[j][2], re = r1own[j][3];
                int fp = R1_NONE;
                for (long long base = rb; base < re; base += 4 * WG) {
                    int w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const long long e = base + k * WG + threadIdx.x;
                        w[k] = e < re ? colidx[e] : -1;
                    }
                    int mine = R1_NONE;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (mine == R1_NONE && w[k] >= 0 && w[k] != rv && beats(rule, rowptr, w[k], rv, re - rb))
                            mine = (int)(base + k * WG + threadIdx.x - rb);
                    if (mine != R1_NONE) atomicMin(&r1pos[slot], mine);
                    // the next step's slot was last read before the previous barrier
                    const int nxt = slot == 2 ? 0 : slot + 1;
                    if (threadIdx.x == 0) r1pos[nxt] = R1_NONE;
                    __syncthreads();
                    fp = r1pos[slot];
                    slot = nxt;
                    if (fp != R1_NONE) break;
                }
                if ((int)threadIdx.x == own) {
                    by = fp != R1_NONE ? colidx[rb + fp] : -1;
                    lose = by >= 0;
                    pend = false;
                }
            }
        }
        if (vv < n) {
            const int v = (int)vv;
            if (hint && rflag) {
                // wake flags: the hint of a short loser names its class, a long loser's hint
                // carries FLAG, a winner's is cleared: a hint without FLAG names a sleeper
                if (!lose) {
                    hint[v] = -1;
                } else if (end - beg <= WAKE_DEG) {
                    const bool big = rowptr[by + 1] - rowptr[by] > WAKE_DEG;
                    hint[v] = big ? (by | FLAG) : by;
                    aflag[v] = big;
                } else {
                    hint[v] = by | FLAG;
                }
            } else if (lose && hint) {
                hint[v] = by;
            }
            if (lose) {
                X[v] = jp ? 0 : (FLAG | 1 | (rflag && end - beg > WAKE_DEG ? BIG : 0));
                bkt = bucket_of(end - beg, tiles, twave, tsplit);
                if (rflag && bkt < NTILE) bkt = -1;      // wake flags: not listed
                if (llen && bkt >= NTILE && bkt < BSPLIT) llen[v] = -1;   // live list not built yet
                if (bkt == BSPLIT) {
                    // split rows are few: one queue slot and one chunk range per vertex
                    const int nch = split_chunks(end - beg);
                    const int p = atomicAdd(&ctl->cnt[1][BSPLIT], 1);
                    const int cs = atomicAdd(&ctl->ccnt[1], nch);
                    wl1[seg[BSPLIT] + p] = v;
                    cstart1[p] = cs;
                    for (int k = 0; k < nch; ++k) owner1[cs + k] = p;
                    if (llen) {
                        // the round-1 chunk range doubles as the hub's stable slot range
                        // for its per-chunk live-list lengths
                        llen[v] = cs;
                        for (int k = 0; k < nch; ++k) clen[cs + k] = -1;
                    }
                    if (crec1)
                        for (int k = 0; k < nch; ++k) crec1[cs + k] = make_int4(p, v, k, cs + k);
                    bkt = -1;
                }
            } else {
                X[v] = 1;
                out[v] = 0;
                if (srnd) srnd[v] = 1;
                winpush = F != nullptr && end > beg;
                wbeg = beg;
                wend = end;
            }
        }
        // round-1 winners push colour 1, the whole wavefront over their concatenated rows
        if (F != nullptr) push_rows_wave(P, winpush, (int)vv, 1, wbeg, wend);
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
    if (lb1) {
        // one wavefront per bucket runs its look-back (wavefront w: buckets w, w + WAVES);
        // every count is published before any walk starts
        for (int b = wv; b < NB; b += WAVES) {
            int tot = 0;
            for (int w = 0; w < WAVES; ++w) tot += wcnt[w][b];
            lookback_publish(lb1 + (size_t)b * gridDim.x, unit, tot);
        }
        for (int b = wv; b < NB; b += WAVES) {
            int tot = 0;
            for (int w = 0; w < WAVES; ++w) tot += wcnt[w][b];
            const int base = lookback_walk(lb1 + (size_t)b * gridDim.x, unit, tot, &ctl->err);
            if (lane == 0) {
                const int pos = tot ? atomicAdd(&ctl->cnt[1][b], tot) : 0;
                int bs = base >= 0 ? base : pos;   // a walk that gave up takes the unordered slot
                for (int w = 0; w < WAVES; ++w) { wbase[w][b] = bs; bs += wcnt[w][b]; }
            }
        }
    } else if (threadIdx.x < NB) {
        const int b = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += wcnt[w][b];
        int base = tot ? atomicAdd(&ctl->cnt[1][b], tot) : 0;
        for (int w = 0; w < WAVES; ++w) { wbase[w][b] = base; base += wcnt[w][b]; }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int* dst = wl1 + seg[b] + wbase[wv][b];
        for (int k = lane; k < cnt[b]; k += 64) dst[k] = buf[wv][b][k];
    }
}


__global__ __launch_bounds__(WG) void k_round1(int n, const int* __restrict__ rowptr,
                                               const int* __restrict__ colidx, int* X, int* out,
                                               int* wl1, Ctl* ctl, int sorted, int twave, int tsplit,
                                               Seg seg, int* cstart1, int* owner1, unsigned* F, int nnz,
                                               int rule, int jp, int* hint, int* llen, int* clen,
                                               unsigned long long* lb1, int fbytes, unsigned char* dirty,
                                               unsigned char* rflag, unsigned char* aflag, int* srnd,
                                               unsigned long long* Fs, unsigned char* Fq, int4* crec1, int tiles) {
    round1_body(n, rowptr, colidx, X, out, wl1, ctl, sorted, twave, tsplit, seg.s, cstart1, owner1, F, nnz,
                rule, jp, hint, llen, clen, lb1, fbytes, dirty, rflag, aflag, srnd, Fs, Fq, crec1, tiles);
}

// Flag-scanning conflict test of the vertices of at most WAKE_DEG arcs, run by block
// bid of nblk such blocks: every wavefront scans the test flags of its vpw
// vertices and tests the flagged ones.  A wavefront that tests a vertex stores the
// round number (every writer stores the same).
template <bool C>
__device__ __forceinline__ void detect_flags_phase(const RoundArgs& a, int* ids, int* slot, int bid, int nblk,
                                                   int& cmax, long long* red64) {
    long long nb = 0;          // bytes moved (counted only on request)
    bool any = false;
    const long long nwv = (long long)nblk * WAVES;
    const int k = a.vpw / 64;
    for (long long wid = (long long)bid * WAVES + (threadIdx.x >> 6); wid * a.vpw < a.n; wid += nwv) {
        const long long v0 = wid * a.vpw;
        const int cnt = flag_compact(load_flags(a.aflag, v0, k), (int)v0, k, ids);
        if (C) nb += k;
        if (cnt) {
            any = true;
            test_flagged<C>(a, ids, cnt, slot, cmax, nb);
        }
    }
    if (any && __lane_id() == 0) a.ctl->rounds = wround_of(a);
    if (C) {
        const long long t = block_sum64(nb, red64);
        if (threadIdx.x == 0 && t) atomicAdd(&a.ubytes[1], (unsigned long long)t);
    }
}

// Conflict test of a round (Sec. 3, ConflictResolve; see detect_phase), one launch for
// every degree bucket (with wake flags only the rows longer than WAKE_DEG are on the
// worklists).
// Four workgroups per CU: the conflict test needs about 104 VGPRs, and with six per CU
// the compiler kept 80 and spilled 108 bytes per lane to scratch (R-MAT scale 23:
// 40.3 -> 39.7 ms with four).  Its grid is at most this many blocks per CU, so that every
// block is resident at once.
constexpr int DETECT_PER_CU = 4;

template <bool W>
__global__ __launch_bounds__(WG, DETECT_PER_CU) void k_detect(RoundArgs a) {
    __shared__ RoundLds s;
    __shared__ int boff[NB + 1];
    if (threadIdx.x == 0) {
        if (a.dev_plan) {
            int cnt[NB];
            queue_sizes(a.ctl, a.par_in, cnt);
            // the round index: counted by the FirstFit phase, so it is fixed here
            device_plan(cnt, gridDim.x, boff, a.ctl->pround);
        } else {
            for (int k = 0; k <= NB; ++k) boff[k] = a.boff[k];
        }
    }
    __syncthreads();
    int cmax = 0;
    detect_phase<W>(a, s, blockIdx.x, boff, cmax);
    cmax = block_max(cmax, s.red);
    // with wake flags a colour at or below the current maximum needs no device atomic
    if (threadIdx.x == 0 && cmax > 0 && (!W || cmax > ld_agent(&a.ctl->maxcolor)))
        atomicMax(&a.ctl->maxcolor, cmax);
}

// Flag-scanning conflict test of a round with wake flags (the rows longer than WAKE_DEG,
// if any, are tested by k_detect<true> in a launch of their own: measured faster than
// one launch for both, whose register allocation suits neither).
template <bool C>
__global__ __launch_bounds__(WG) void k_detect_flags(RoundArgs a) {
    __shared__ int ids[WAVES][VPW];
    __shared__ int slot[WAVES][64];
    __shared__ int red[WAVES];
    __shared__ long long red64[WAVES];
    const int wv = threadIdx.x >> 6;
    if (a.ctl->rounds < wround_of(a) - 1) return;    // past the end of the colouring
    int cmax = 0;
    detect_flags_phase<C>(a, ids[wv], slot[wv], blockIdx.x, gridDim.x, cmax, red64);
    cmax = block_max(cmax, red);
    if (threadIdx.x == 0 && cmax > ld_agent(&a.ctl->maxcolor)) atomicMax(&a.ctl->maxcolor, cmax);
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

// One graph of a multi-graph call: device pointers, its place in the union and sizes.
struct MultiDesc {
    const int* rowptr;
    const int* colidx;
    int* colors;
    long long voff;
    long long eoff;
    int n;
    int pad;
    long long nnz;
};

// Copies graph blockIdx.y into the union CSR with ids shifted by its vertex offset and
// row offsets shifted by its arc offset; the last graph also writes rowptr[N].
__global__ __launch_bounds__(WG) void k_concat(const MultiDesc* __restrict__ d, int G, int* urowptr, int* ucolidx,
                                               long long N, long long E, Ctl* ctl) {
    const int g = blockIdx.y;
    const MultiDesc m = d[g];
    const long long stride = (long long)gridDim.x * WG;
    const long long t0 = (long long)blockIdx.x * WG + threadIdx.x;
    if (t0 == 0 && (m.rowptr[0] != 0 || m.rowptr[m.n] != m.nnz)) atomicOr(&ctl->err, ERR_MULTI);
    for (long long i = t0; i < m.n; i += stride) urowptr[m.voff + i] = m.rowptr[i] + (int)m.eoff;
    for (long long j = t0; j < m.nnz; j += stride) ucolidx[m.eoff + j] = m.colidx[j] + (int)m.voff;
    if (g == G - 1 && t0 == 0) urowptr[N] = (int)E;
}

// Copies each graph's colours from the union output to its own buffer.
__global__ __launch_bounds__(WG) void k_scatter(const MultiDesc* __restrict__ d, const int* __restrict__ ucolors) {
    const MultiDesc m = d[blockIdx.y];
    for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < m.n; i += (long long)gridDim.x * WG)
        m.colors[i] = ucolors[m.voff + i];
}

// Batched validation: voff[0] == 0, non-decreasing, voff[G] == n_total, and every
// arc of graph g stays inside graph g.  The graph checks are a grid-stride loop over
// g.  The arc checks are spread over the whole grid whatever the graph sizes: every
// wavefront takes chunks of VB_CHUNK consecutive arc positions, finds the graph that
// owns the chunk's first position (the last g whose first arc rowptr[voff[g]] is at or
// before it) by binary search, and steps to the next graph wherever a position passes
// the current graph's last arc.  Runs after the row pass accepted rowptr; the voff
// entries it follows are clamped to [0, n_total], so a malformed voff (which fails the
// graph checks) still keeps every read in bounds.
constexpr int VB_CHUNK = 4096;

__global__ __launch_bounds__(WG) void k_validate_batch(int G, int n_total, const long long* __restrict__ voff,
                                                       const int* __restrict__ rowptr,
                                                       const int* __restrict__ colidx, Ctl* ctl) {
    // rowptr already failed validation: its entries are not trustworthy bounds
    if (ctl->err) return;
    int bad = 0;
    const long long nnz = rowptr[n_total];
    const long long nthr = (long long)gridDim.x * WG;
    for (long long g = (long long)blockIdx.x * WG + threadIdx.x; g < G; g += nthr) {
        const long long v0 = voff[g], v1 = voff[g + 1];
        if ((g == 0 && v0 != 0) || v0 < 0 || v0 > n_total || v1 < v0 || v1 > n_total || (g == G - 1 && v1 != n_total))
            bad = 1;
    }
    const int lane = __lane_id();
    const long long nw = (long long)gridDim.x * WAVES;
    for (long long c = (long long)blockIdx.x * WAVES + (threadIdx.x >> 6); c * VB_CHUNK < nnz; c += nw) {
        const long long e0 = c * VB_CHUNK, e1 = min(e0 + VB_CHUNK, nnz);
        int lo = 0, hi = G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const long long vm = min(max(voff[mid], 0ll), (long long)n_total);
            if (rowptr[vm] <= e0) lo = mid;
            else hi = mid - 1;
        }
        int g = lo;
        long long v0 = min(max(voff[g], 0ll), (long long)n_total);
        long long v1 = min(max(voff[g + 1], 0ll), (long long)n_total);
        long long gend = rowptr[v1];
        for (long long e = e0 + lane; e < e1; e += 64) {
            while (e >= gend && g < G - 1) {
                ++g;
                v0 = v1;
                v1 = min(max(voff[g + 1], 0ll), (long long)n_total);
                gend = rowptr[v1];
            }
            const int w = colidx[e];
            if (w < v0 || w >= v1) bad = 1;
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->err, ERR_BATCH);
}

}  // namespace csrcolor
