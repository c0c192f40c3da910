// Wake flags: the rounds of Sec. 3.1 (Algorithm Data-GC, id rule) without re-testing
// the requeued vertices whose verdict cannot have changed.
//
// Under the id rule with conflict hints, a requeued vertex v remembers the neighbour h
// that beat it: h < v, h uncoloured, with v's tentative colour.  Next round v loses to
// h again unless one of the two tentative colours changed, and a tentative colour only
// changes when a neighbour settles with exactly that colour (FirstFit's smallest free
// colour moves only when that very colour becomes forbidden).  So each round:
//   * a winner that pushes colour c to a neighbour u holding tentative colour c sets
//     u's recolour flag;
//   * FirstFit runs only over the vertices whose recolour flag is set; each of them
//     gets its test flag, and so does every uncoloured higher neighbour w whose hint is
//     the recoloured vertex;
//   * the conflict test runs only over the vertices whose test flag is set; a loser
//     records its hint and clears its flag (it sleeps), a winner settles and pushes.
// Every sleeping vertex keeps its tentative colour and loses to its hint, the verdict
// the full round would give, so the colouring and the rounds are those of the paper's
// method.  If h settles, it pushes its colour (= v's) to v, so v is recoloured.
// Waking reads the row of the recoloured vertex, so only short rows may hold sleepers:
// a requeued vertex whose hint has more than WAKE_DEG arcs (the hint then carries FLAG)
// is awake and keeps its test flag; a vertex of more than WAKE_DEG arcs never sleeps
// and stays on the degree-bucket worklists of the classic rounds.
//
// The flags are bytes, one per vertex, written with plain stores (every writer stores
// the same value), and each round's kernels find their vertices by a dense, coalesced
// scan of the flag bytes: VPW vertices per wavefront, a few bytes per vertex and
// round, instead of device-wide list counters whose atomics would serialise.
#pragma once

#include "sgr_device.h"
#include "sgr_round.h"

namespace csrcolor {

constexpr int VPW = 512;   // most vertices per wavefront in the flag scans (8 per lane)
constexpr int TQ = 2;      // quads of colidx per lane and pass in the conflict test
constexpr int WQ = 2;      // the same in the walk that wakes sleepers

// Smallest free colour of v from its push-mode flags: the first clear flag at or after
// position rowptr[v] + v (flags before it count as set); one exists within deg(v) + 1.
__device__ __forceinline__ int first_free(const RoundArgs& a, int beg, int v, int& words) {
    const long long bit = (long long)beg + v;
    long long pos;
    long long k0;
    if (a.pushff == 2) {
        long long k = bit >> 2;
        k0 = k;
        unsigned w = a.F[k] | ((1u << (8 * (bit & 3))) - 1u);
        unsigned z = (w - 0x01010101u) & ~w & 0x80808080u;
        while (z == 0) {
            w = a.F[++k];
            z = (w - 0x01010101u) & ~w & 0x80808080u;
        }
        pos = k * 4 + (__ffs(z) - 1) / 8;
        words = (int)(k - k0) + 1;
    } else {
        long long k = bit >> 5;
        k0 = k;
        unsigned w = a.F[k] | ((1u << (bit & 31)) - 1u);
        while (w == 0xffffffffu) w = a.F[++k];
        pos = k * 32 + __ffs(~w) - 1;
        words = (int)(k - k0) + 1;
    }
    return (int)(pos - bit + 1);
}

// Flag bytes of the wavefront's vertices v0 .. v0 + 64k - 1, k (1, 2, 4 or 8) per lane
// (the arrays are padded with zeros to a whole number of VPW).
__device__ __forceinline__ unsigned long long load_flags(const unsigned char* fl, long long v0, int k) {
    const int lane = __lane_id();
    if (k == 8) return reinterpret_cast<const unsigned long long*>(fl + v0)[lane];
    if (k == 4) return reinterpret_cast<const unsigned*>(fl + v0)[lane];
    if (k == 2) return reinterpret_cast<const unsigned short*>(fl + v0)[lane];
    return fl[v0 + lane];
}

// Lists the vertices whose flag byte is set (lane l holds the bytes of vertices
// v0 + kl .. v0 + kl + k - 1 in f) in ids, in id order; returns their number.  Every
// lane must call.
__device__ __forceinline__ int flag_compact(unsigned long long f, int v0, int k, int* ids) {
    const int lane = __lane_id();
    unsigned m = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < k && ((f >> (8 * j)) & 0xffu)) m |= 1u << j;
    int tot;
    int pos = wave_excl(__popc(m), tot);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (m >> j & 1) ids[pos++] = v0 + k * lane + j;
    __builtin_amdgcn_wave_barrier();
    return tot;
}

// The wavefront walks the rows of its recoloured vertices (lane l: row [beg, end) of
// u when `on`; at most WAKE_DEG arcs) as one concatenation of 16-byte quads, like
// push_rows_wave, and sets the test flag of every neighbour w > u whose hint is u
// (without FLAG: w sleeps).  Every lane must call.
template <bool C>
__device__ __forceinline__ void wake_children(const RoundArgs& a, bool on, int u, int beg, int end,
                                              long long& nb) {
    const int lane = __lane_id();
    const int mis = (int)((reinterpret_cast<uintptr_t>(a.colidx) >> 2) & 3);
    const int nq = on && end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
    int incl = nq;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    // WQ quads per lane per pass (items lane, 64 + lane, ...), loads in flight together
    for (int base = 0; base < total; base += 64 * WQ) {
        int q[WQ], uj[WQ], bj[WQ], ej[WQ];
#pragma unroll
        for (int t = 0; t < WQ; ++t) {
            const int item = base + 64 * t + lane;
            int j = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                if (__shfl(incl, j + step - 1, 64) <= item) j += step;
            }
            q[t] = item - (__shfl(incl, j, 64) - __shfl(nq, j, 64));
            uj[t] = __shfl(u, j, 64);
            bj[t] = __shfl(beg, j, 64);
            ej[t] = __shfl(end, j, 64);
        }
        int w[WQ][4];
#pragma unroll
        for (int t = 0; t < WQ; ++t) {
            if (base + 64 * t + lane < total) {
                load_quad(a.colidx, a.nnz, bj[t], ej[t], q[t], w[t]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) w[t][k] = -1;
            }
        }
        int h[WQ][4];
#pragma unroll
        for (int t = 0; t < WQ; ++t)
#pragma unroll
            for (int k = 0; k < 4; ++k) h[t][k] = w[t][k] > uj[t] ? a.hint[w[t][k]] : -1;
        // a hint equal to u (no FLAG) is held only by an uncoloured vertex of at most
        // WAKE_DEG arcs: settling clears a hint and long rows' hints carry FLAG
#pragma unroll
        for (int t = 0; t < WQ; ++t)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (w[t][k] > uj[t] && h[t][k] == uj[t]) a.aflag[w[t][k]] = 1;
        if (C) {
            // colidx entries, hints of the higher ones, the sleepers' test flags
#pragma unroll
            for (int t = 0; t < WQ; ++t)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    nb += (w[t][k] >= 0 ? 4 : 0) + (w[t][k] > uj[t] ? 4 : 0) +
                          (w[t][k] > uj[t] && h[t][k] == uj[t] ? 1 : 0);
        }
    }
}

// FirstFit of a round with wake flags: every wavefront scans the recolour flags of its
// vpw vertices, recolours the flagged ones, sets their test flags (short rows; longer
// ones are on the worklists) and those of their sleepers.  Block 0 also clears the
// worklist counters the conflict test of the round fills.
template <bool C>
__global__ __launch_bounds__(WG) void k_wassign(RoundArgs a) {
    __shared__ int ids[WAVES][VPW];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    // a previous round that tested nothing ended the colouring: rounds launched past the
    // end return at once.  Rounds replayed from a captured graph: this kernel advances the
    // device round count (its first thread), so its other blocks read the old or the new
    // count; taking the count as read before the advance, the test below fires at most one
    // round late (never early), and the kernels after this one read the advanced count
    int wround = a.wround;
    if (a.wround_dev) {
        wround = __hip_atomic_load(a.wround_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(const_cast<int*>(a.wround_dev), 1);
    }
    if (a.ctl->rounds < wround - 1) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NB; ++k) {
            a.ctl->cnt[a.par_out][k] = 0;
            a.ctl->dyn[1][k] = 0;
        }
        a.ctl->ccnt[a.par_out] = 0;
        a.ctl->nsettled = 0;
        a.ctl->pround += 1;
    }
    const long long nwv = (long long)gridDim.x * WAVES;
    const int k = a.vpw / 64;
    long long nb = 0;          // bytes moved (counted only on request)
    for (long long wid = (long long)blockIdx.x * WAVES + wv; wid * a.vpw < a.n; wid += nwv) {
        const long long v0 = wid * a.vpw;
        const int cnt = flag_compact(load_flags(a.rflag, v0, k), (int)v0, k, ids[wv]);
        if (C) nb += k;
        for (int i0 = 0; i0 < cnt; i0 += 64) {
            const int i = i0 + lane;
            const int u = i < cnt ? ids[wv][i] : -1;
            // every read of the lane (its row bounds, colour word, mask, then the walk
            // over its row) comes before its writes: a read issued after a write would
            // wait for that write as well
            int beg = 0, end = 0, x = 1;
            unsigned long long fs = 0;
            if (u >= 0) {
                beg = a.rowptr[u];
                end = a.rowptr[u + 1];
                x = a.X[u];
                fs = a.Fs[u];          // used by short rows only
                if (C) nb += 13;
            }
            reads_done(beg ^ end ^ x ^ (int)fs ^ (int)(fs >> 32));
            const bool on = x < 0;     // flagged vertices are uncoloured; kept as a guard
            int c = 0;
            if (on) {
                if (x & BIG) {
                    int words = 0;
                    c = first_free(a, beg, u, words);
                    if (C) nb += 4 * words;
                } else {
                    // a short row's forbidden colours in one mask: the smallest free colour
                    // is at most 62, so the lowest clear bit exists
                    c = __ffsll((long long)~fs);
                    if (C) nb += 8;
                }
            }
            const bool small = on && end - beg <= WAKE_DEG;
            wake_children<C>(a, small, u, beg, end, nb);
            if (u >= 0) a.rflag[u] = 0;
            if (on) {
                a.X[u] = (x & BIG) | FLAG | c;
                if (C) nb += 4;
            }
            if (small) {
                a.aflag[u] = 1;
                if (C) nb += 1;
            }
        }
    }
    if (C) {
        __shared__ long long red64[WAVES];
        const long long t = block_sum64(nb, red64);
        if (threadIdx.x == 0 && t) atomicAdd(&a.ubytes[0], (unsigned long long)t);
    }
}

// Conflict test of the flagged vertices of one wavefront's range (ids, cnt; all of at
// most WAKE_DEG arcs).  Their rows are walked as one concatenation of quads; a lower
// neighbour with the same tentative colour requeues the vertex, and the largest such
// neighbour becomes its hint (slot: per-vertex LDS verdicts).  A loser sleeps unless
// its hint is long; a winner settles and pushes its colour.  Every lane must call.
template <bool C>
__device__ __forceinline__ void test_flagged(const RoundArgs& a, const int* ids, int cnt, int* slot, int& cmax,
                                             long long& nb) {
    const int lane = __lane_id();
    PushCtx P = push_ctx<true>(a);
    if (C) P.nbytes = &nb;
    const int mis = (int)((reinterpret_cast<uintptr_t>(a.colidx) >> 2) & 3);
    for (int i0 = 0; i0 < cnt; i0 += 64) {
        const int i = i0 + lane;
        int v = i < cnt ? ids[i] : -1;
        int cv = 0, beg = 0, end = 0, hv = -1;
        if (v >= 0) {
            const int x = a.X[v];
            hv = a.hint[v];
            beg = a.rowptr[v];
            end = a.rowptr[v + 1];
            cv = x & CMASK;
            if (x > 0) {               // guard: a flagged vertex is uncoloured
                a.aflag[v] = 0;
                v = -1;
            }
        }
        // an awake vertex (long hint) usually still loses to it: then no row walk
        const bool held = v >= 0 && hv < 0 && hv != -1 && (a.X[hv & IDMASK] & CMASK) == cv;
        if (C && v >= 0) nb += 16 + (hv < 0 && hv != -1 ? 4 : 0);   // colour, hint, rowptr pair, hint's colour
        // verdict slot: 0 = no conflict, else 1 + (2 * neighbour + 1 if it is long); the
        // largest conflicting neighbour wins the atomic maximum
        slot[lane] = held ? (int)(2u * (unsigned)(hv & IDMASK) + 2u) : 0;
        __builtin_amdgcn_wave_barrier();
        const int nq = v >= 0 && !held && end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
        int incl = nq;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        const int total = __shfl(incl, 63, 64);
        // TQ quads per lane per pass (items lane, 64 + lane, ...), their loads and colour
        // gathers in flight together; the quads of the last pass stay in registers: when
        // one pass covers every row, the winners push from them without reading their rows
        // again
        int w[TQ][4];
        int j[TQ], vj[TQ], cj[TQ];
#pragma unroll
        for (int u = 0; u < TQ; ++u) {
            j[u] = 0;
            vj[u] = -1;
            cj[u] = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) w[u][k] = -1;
        }
        for (int base = 0; base < total; base += 64 * TQ) {
            int q[TQ], bj[TQ], ej[TQ];
#pragma unroll
            for (int u = 0; u < TQ; ++u) {
                const int item = base + 64 * u + lane;
                int jj = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    if (__shfl(incl, jj + step - 1, 64) <= item) jj += step;
                }
                j[u] = jj;
                q[u] = item - (__shfl(incl, jj, 64) - __shfl(nq, jj, 64));
                vj[u] = __shfl(v, jj, 64);
                cj[u] = __shfl(cv, jj, 64);
                bj[u] = __shfl(beg, jj, 64);
                ej[u] = __shfl(end, jj, 64);
            }
#pragma unroll
            for (int u = 0; u < TQ; ++u) {
                if (base + 64 * u + lane < total) {
                    load_quad(a.colidx, a.nnz, bj[u], ej[u], q[u], w[u]);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) w[u][k] = -1;
                }
            }
            int x[TQ][4];
#pragma unroll
            for (int u = 0; u < TQ; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) x[u][k] = (w[u][k] >= 0 && w[u][k] < vj[u]) ? a.X[w[u][k]] : 0;
#pragma unroll
            for (int u = 0; u < TQ; ++u) {
                unsigned found = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((x[u][k] & CMASK) == cj[u])
                        found = max(found, 2u * (unsigned)w[u][k] + ((x[u][k] & BIG) ? 2u : 1u));
                if (found) atomicMax(reinterpret_cast<unsigned*>(&slot[j[u]]), found);
                if (C) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        nb += (w[u][k] >= 0 ? 4 : 0) + (w[u][k] >= 0 && w[u][k] < vj[u] ? 4 : 0);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        const unsigned e = (unsigned)slot[lane];
        const bool win = v >= 0 && e == 0;
        if (v >= 0 && !held) {
            if (e) {
                const int h = (int)((e - 1) >> 1);
                const bool big = ((e - 1) & 1) != 0;
                a.hint[v] = big ? (h | FLAG) : h;
                if (!big) a.aflag[v] = 0;          // asleep until woken
                if (C) nb += 4 + (big ? 0 : 1);
            } else {
                settle<true>(a, v, cv, cmax);
                a.aflag[v] = 0;
                a.hint[v] = -1;                    // a settled vertex is nobody's sleeper
                if (C) nb += 17;
            }
        }
        if (total <= 64 * TQ) {
            // item lane (+ 64 u): its quad belongs to vertex j[u], a winner when no conflict
            // was found
            PushCtx Q = P;
            Q.loaded = true;
            // every neighbour's colour word is read before any flag is written
            bool go[TQ];
            PushRead r[TQ][4];
            int all = 0;
#pragma unroll
            for (int u = 0; u < TQ; ++u) {
                go[u] = 64 * u + lane < total && slot[j[u]] == 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    r[u][k].a = 1;
                    r[u][k].b = 0;
                    if (go[u] && w[u][k] >= 0 && w[u][k] != vj[u]) r[u][k] = push_read(Q, w[u][k]);
                    all |= r[u][k].a | r[u][k].b;
                }
            }
            reads_done(all);
#pragma unroll
            for (int u = 0; u < TQ; ++u) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (go[u] && w[u][k] >= 0 && w[u][k] != vj[u]) push_write(Q, w[u][k], cj[u], r[u][k]);
            }
        } else {
            push_rows_wave(P, win, v, cv, beg, end);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-round statistics from the settling rounds: bins[s-1] += 1 and abins[s-1] +=
// deg(v) for every vertex v that settled in round s <= cap (the caller turns them
// into worklist sizes and arcs).  Rounds up to HROUNDS are first summed in LDS per
// block (one device atomic per block and round), later ones directly.
constexpr int HROUNDS = 1024;
__global__ __launch_bounds__(WG) void k_round_hist(int n, const int* __restrict__ rowptr, const int* srnd,
                                                   long long* bins, long long* abins, int cap) {
    __shared__ unsigned hb[HROUNDS];
    __shared__ unsigned long long ha[HROUNDS];
    for (int i = threadIdx.x; i < HROUNDS; i += WG) {
        hb[i] = 0;
        ha[i] = 0;
    }
    __syncthreads();
    for (long long v = (long long)blockIdx.x * WG + threadIdx.x; v < n; v += (long long)gridDim.x * WG) {
        const int s = srnd[v];
        if (s < 1 || s > cap) continue;
        const unsigned long long d = (unsigned long long)(rowptr[v + 1] - rowptr[v]);
        if (s <= HROUNDS) {
            atomicAdd(&hb[s - 1], 1u);
            atomicAdd(&ha[s - 1], d);
        } else {
            atomicAdd((unsigned long long*)&bins[s - 1], 1ull);
            atomicAdd((unsigned long long*)&abins[s - 1], d);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HROUNDS && i < cap; i += WG) {
        if (hb[i]) {
            atomicAdd((unsigned long long*)&bins[i], (unsigned long long)hb[i]);
            atomicAdd((unsigned long long*)&abins[i], ha[i]);
        }
    }
}

}  // namespace csrcolor
