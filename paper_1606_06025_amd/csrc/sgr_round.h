// Round phases: FirstFit (k_assign) and conflict test + clearing + compaction (the
// phase run by k_detect), one launch each per round, every degree bucket in the same
// grid.
//
// Cost model that shapes them: on gfx950 a wave64 vector-memory instruction costs
// the compute unit's address unit about the same whatever its lanes do, so the
// kernels minimise VMEM instructions per arc:
//   * per-vertex metadata (worklist entry, rowptr pair, own colour) is loaded once,
//     one lane per vertex, and handed to the lanes that need it by cross-lane moves;
//   * row entries are read as aligned 16-byte quads (four arcs per lane per load);
//   * one neighbour-colour gather per arc is the only per-arc instruction left.
#pragma once

#include "sgr_device.h"

namespace csrcolor {

struct RoundLds {
    union {
        int lbuf[WAVES * WAVE_CAP];   // detect: per-wavefront loser buffers
        unsigned ovf[WAVES * OVW];    // assign, wavefront bucket: overflow colour bitmaps
        unsigned bm[BMW];             // assign, workgroup bucket: colour window bitmap
    };
    int res[WAVES * 64];              // per-wavefront staging of per-vertex results
    int idx[WAVES * 128];             // detect tiles: per-wavefront list of the entries still to be tested
    int res2[WAVES * 128];            // detect tiles: their verdicts
    int wcnt[WAVES];
    int wbase[WAVES];
    int red[WAVES];
    long long red64[WAVES];
    int sh[4];
    int lpre[WAVES];                  // live lists: per-wavefront kept counts of a block scan
    int lsh[4];                       // live lists: block-uniform verdicts of a split chunk
    int wbuf[WAVES * 4 * 128];        // detect stream: per-wavefront winners staged for their pushes
};

// Bucket of block `bid` under the partition boff, its index j inside the bucket and
// the bucket's block count.  Blocks are dispatched round-robin over the 8 XCDs, so
// the index is remapped to give every XCD one contiguous slice of the bucket's
// worklist: neighbouring vertices then share an L2.
__device__ __forceinline__ void block_bucket(const int* boff, int bid, int& b, int& j, int& nbk) {
    b = 0;
#pragma unroll
    for (int k = 1; k < NB; ++k)
        if (bid >= boff[k]) b = k;
    const int s0 = boff[b];
    nbk = boff[b + 1] - s0;
    const int jj = bid - s0;
    if (nbk >= 8) {
        const int x = (s0 + jj) & 7;          // XCD of this block
        int before = 0;                       // blocks of the range on XCDs < x
        for (int y = 0; y < x; ++y) {
            const int j0 = (y - s0) & 7;
            before += nbk > j0 ? (nbk - j0 + 7) >> 3 : 0;
        }
        const int j0 = (x - s0) & 7;
        j = before + ((jj - j0) >> 3);
    } else {
        j = jj;
    }
}

// Per-bucket cost weights (time per queued unit: a worklist vertex, or a chunk of a
// split row) and the most blocks a bucket can use per unit, shared by the host plan
// and the device plan.  The weights follow the block time per unit measured on MI355X
// on R-MAT scale 23: live lists and hints make the tests cost per vertex rather than
// per arc.  In the first rounds (0-based round index r <= 2) every long row and chunk
// is read for the first time (vertex of at most 61 arcs : 62-1024 arcs : 1025-2048
// arcs : 2048-arc chunk about 0.16 : 0.6 : 1.3-2.3 : 1.5 block-us); from r = 10 on
// the lists are built and a chunk costs about what a wavefront-bucket vertex does
// (1 : 1.8 : 1); in between the weights move linearly.
__host__ __device__ inline int plan_cost(int b, int r) {
    constexpr int fresh[NB] = {50, 60, 60, 60, 200, 600, 450};
    constexpr int steady[NB] = {50, 60, 60, 60, 200, 380, 210};
    const int f = r <= 2 ? 8 : r >= 10 ? 0 : 10 - r;     // eighths of the way back to fresh
    return steady[b] + (fresh[b] - steady[b]) * f / 8;
}
__host__ __device__ inline int plan_units_per_block(int b) {
    constexpr int u[NB] = {WG, WG, WG, WG, WAVES, WAVES, WAVES};
    return u[b];
}

// Partition of nblk blocks over the buckets for queue sizes cnt[] (chunks for the
// split bucket) in 0-based round r: one block per non-empty bucket, the rest in
// proportion to the estimated work, capped by what a bucket can use.  Integer arithmetic only,
// so every block that evaluates it gets the same answer.
__device__ __forceinline__ void device_plan(const int* cnt, int nblk, int* boff, int r) {
    long long tot = 0;
    int nz = 0;
    for (int b = 0; b < NB; ++b) {
        tot += (long long)cnt[b] * plan_cost(b, r);
        nz += cnt[b] > 0;
    }
    const long long rem = nblk > nz ? nblk - nz : 0;
    boff[0] = 0;
    for (int b = 0; b < NB; ++b) {
        int nb = 0;
        if (cnt[b] > 0) {
            const long long extra = tot > 0 ? rem * cnt[b] * plan_cost(b, r) / tot : 0;
            const int useful = (cnt[b] + plan_units_per_block(b) - 1) / plan_units_per_block(b);
            nb = (int)min((long long)useful, 1 + extra);
        }
        boff[b + 1] = boff[b] + nb;
    }
}

// Quad q of row [beg, end): the q-th 16-byte aligned group of four colidx entries,
// counted from the group holding colidx[beg] (alignment of the absolute address).
// Entries outside the row come back as -1.  The 16-byte load is used only when the
// whole group lies inside colidx[0, nnz); otherwise entries are read one by one.
__device__ __forceinline__ void load_quad(const int* __restrict__ colidx, int nnz, int beg, int end, int q,
                                          int w[4]) {
    const int mis = (int)((reinterpret_cast<uintptr_t>(colidx) >> 2) & 3);
    const int qs = ((beg + mis) & ~3) - mis + 4 * q;
    if (qs >= end) {
        w[0] = w[1] = w[2] = w[3] = -1;
        return;
    }
    if (qs >= 0 && qs + 4 <= nnz) {
        const int4 t = *reinterpret_cast<const int4*>(colidx + qs);
        w[0] = t.x;
        w[1] = t.y;
        w[2] = t.z;
        w[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = qs + k;
            w[k] = (e >= 0 && e < nnz) ? colidx[e] : -1;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (qs + k < beg || qs + k >= end) w[k] = -1;
}

// First position (relative to beg) after the quads 0 .. q-1 of src[beg, ...).
__device__ __forceinline__ int quad_end(const int* src, int beg, int q) {
    const int mis = (int)((reinterpret_cast<uintptr_t>(src) >> 2) & 3);
    return ((beg + mis) & ~3) - mis + 4 * q - beg;
}

// Quads of src[beg, end) (0 if the range is empty).
__device__ __forceinline__ int quad_count(const int* src, int beg, int end) {
    const int mis = (int)((reinterpret_cast<uintptr_t>(src) >> 2) & 3);
    return end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
}

// Contiguous slice [wlo, whi) of [lo, hi) for the calling wavefront.
__device__ __forceinline__ void wave_slice(int lo, int hi, int& wlo, int& whi) {
    const int wv = threadIdx.x >> 6;
    const int q = (hi - lo + WAVES - 1) / WAVES;
    wlo = min(hi, lo + wv * q);
    whi = min(hi, wlo + q);
}

// ---------------------------------------------------------------------------
// Push mode: a vertex that settles with colour c sets bit c-1 in the forbidden
// bitmap F of each neighbour (once in its life); FirstFit then reads the vertex's
// own bitmap instead of gathering every neighbour's colour every round.  The bitmap
// of v at round r holds exactly the colours of neighbours settled before round r,
// which is the snapshot FirstFit of Sec. 3 reads, so the colouring is unchanged.
// ---------------------------------------------------------------------------

// `nthr` threads (thread index t) push colour c of v over row [beg, end) together.
__device__ __forceinline__ void push_row_coop(const PushCtx& P, int v, int c, int beg, int end, int t, int nthr) {
    const int nq = ((end - beg) + 3 + 3) / 4 + 1;
    for (int q0 = 0; q0 < nq; q0 += nthr) {
        int w[4];
        load_quad(P.colidx, P.nnz, beg, end, q0 + t, w);
        push_quad(P, w, v, c);
    }
}

// The whole wavefront pushes the colours of its winners: lane l contributes the row
// [beg, end) of vertex v with colour c when `win`.  The rows are concatenated quad by
// quad (a prefix sum over the lanes) and the 64 lanes walk the concatenation, each
// finding its row by a binary search over the prefix, so a wavefront with one long
// or a few short winner rows does not serialise on one lane.  Every lane must call.
__device__ __forceinline__ void push_rows_wave(const PushCtx& P, bool win, int v, int c, int beg, int end) {
    const int lane = __lane_id();
    const int mis = (int)((reinterpret_cast<uintptr_t>(P.colidx) >> 2) & 3);
    const int nq = win && end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
    int incl = nq;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64) {
        const int item = base + lane;
        // j = number of lanes whose inclusive prefix is <= item: the row holding the item
        int j = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            if (__shfl(incl, j + step - 1, 64) <= item) j += step;
        }
        const int q = item - (__shfl(incl, j, 64) - __shfl(nq, j, 64));
        const int vj = __shfl(v, j, 64);
        const int cj = __shfl(c, j, 64);
        const int bj = __shfl(beg, j, 64);
        const int ej = __shfl(end, j, 64);
        if (item < total) {
            int w[4];
            load_quad(P.colidx, P.nnz, bj, ej, q, w);
            push_quad(P, w, vj, cj);
        }
    }
}

// Push context of a round (W: with wake flags).
template <bool W>
__device__ __forceinline__ PushCtx push_ctx(const RoundArgs& a) {
    PushCtx P;
    P.F = a.F;
    P.rowptr = a.rowptr;
    P.colidx = a.colidx;
    P.nnz = a.nnz;
    P.bytes = a.pushff == 2;
    P.dirty = a.dirty;
    P.Fq = W ? nullptr : a.Fq;
    P.X = a.X;
    P.rflag = W ? a.rflag : nullptr;
    P.Fs = W ? a.Fs : nullptr;
    P.all_tentative = false;
    P.nbytes = nullptr;
    P.loaded = false;
    return P;
}
template <bool W>
__device__ __forceinline__ void push_row_coop(const RoundArgs& a, int v, int c, int beg, int end, int t,
                                              int nthr) {
    push_row_coop(push_ctx<W>(a), v, c, beg, end, t, nthr);
}
template <bool W>
__device__ __forceinline__ void push_rows_wave(const RoundArgs& a, bool win, int v, int c, int beg, int end) {
    push_rows_wave(push_ctx<W>(a), win, v, c, beg, end);
}

// Push-mode FirstFit for any bucket: one lane per vertex finds the first clear bit
// of the vertex's bitmap (bits below its start count as set); the scan stops at the
// first clear bit, which exists within deg(v)+1 bits.  Flags are only ever set, so
// the smallest free colour never decreases from one round to the next: the scan
// starts at the vertex's previous tentative colour (every colour below it is taken).
__device__ __forceinline__ void assign_push(const RoundArgs& a, const int* list, int lo, int hi, long long& arcs) {
    // four worklist entries per lane at a time, each step's loads issued together so
    // their latencies overlap
    constexpr int U = 4;
    const int lane = __lane_id();
    const bool bytes = a.pushff == 2;
    int wlo, whi;
    wave_slice(lo, hi, wlo, whi);
    for (int t0 = wlo; t0 < whi; t0 += 64 * U) {
        int v[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int t = t0 + 64 * i + lane;
            v[i] = t < whi ? list[t] : -1;
        }
        bool need[U];
        int beg[U], c0[U];
        if (a.Fq) {
            // small-colour slots: a vertex whose previous colour is at most KQ reads its
            // slot; one above KQ has every colour <= KQ forbidden already and, when none of
            // its flags changed since its last FirstFit, keeps its colour
            int4 sq[U];
            int dq[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
                if (v[i] >= 0) {
                    c0[i] = max(a.X[v[i]] & CMASK, 1);
                    sq[i] = *reinterpret_cast<const int4*>(a.Fq + (size_t)v[i] * KQ);
                    beg[i] = a.rowptr[v[i]];
                    dq[i] = a.dirty ? a.dirty[v[i]] : 1;
                }
            }
#pragma unroll
            for (int i = 0; i < U; ++i) {
                need[i] = false;
                if (v[i] < 0) continue;
                if (c0[i] <= KQ) {
                    const unsigned q4[4] = {(unsigned)sq[i].x, (unsigned)sq[i].y, (unsigned)sq[i].z, (unsigned)sq[i].w};
                    int col = 0;
#pragma unroll
                    for (int k = 3; k >= 0; --k) {
                        const unsigned z = (q4[k] - 0x01010101u) & ~q4[k] & 0x80808080u;
                        if (z) col = 4 * k + (__ffs(z) - 1) / 8 + 1;   // first zero byte of word k
                    }
                    if (col > 0) {
                        a.X[v[i]] = FLAG | col;
                        continue;
                    }
                    c0[i] = KQ + 1;                   // every colour <= KQ is taken
                } else if (dq[i] == 0) {
                    continue;
                }
                need[i] = true;
            }
        } else {
            // a vertex none of whose flags changed since its last FirstFit keeps its colour
#pragma unroll
            for (int i = 0; i < U; ++i) need[i] = v[i] >= 0 && (!a.dirty || a.dirty[v[i]] != 0);
#pragma unroll
            for (int i = 0; i < U; ++i) {
                beg[i] = need[i] ? a.rowptr[v[i]] : 0;
                c0[i] = need[i] ? max(a.X[v[i]] & CMASK, 1) : 1;
            }
        }
        long long wi[U];
        unsigned wd[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const long long bit = (long long)beg[i] + v[i] + c0[i] - 1;
            wi[i] = bytes ? bit >> 2 : bit >> 5;
            wd[i] = need[i] ? a.F[wi[i]] : 0u;
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (!need[i]) continue;
            const long long base = (long long)beg[i] + v[i];   // flag of colour 1
            const long long bit = base + c0[i] - 1;
            long long pos;
            if (bytes) {
                // byte flags: the first zero byte at or after `bit` (bytes before it count as set)
                unsigned w = wd[i] | ((1u << (8 * (bit & 3))) - 1u);
                unsigned z = (w - 0x01010101u) & ~w & 0x80808080u;
                long long k = wi[i];
                while (z == 0) {
                    w = a.F[++k];
                    z = (w - 0x01010101u) & ~w & 0x80808080u;
                }
                pos = k * 4 + (__ffs(z) - 1) / 8;
            } else {
                unsigned w = wd[i] | ((1u << (bit & 31)) - 1u);
                long long k = wi[i];
                while (w == 0xffffffffu) w = a.F[++k];
                pos = k * 32 + __ffs(~w) - 1;
            }
            if (a.dirty) a.dirty[v[i]] = 0;
            a.X[v[i]] = FLAG | (int)(pos - base + 1);
        }
        if (a.st_arcs) {
#pragma unroll
            for (int i = 0; i < U; ++i)
                if (v[i] >= 0) arcs += a.rowptr[v[i] + 1] - a.rowptr[v[i]];
        }
    }
}

// ---------------------------------------------------------------------------
// FirstFit (Sec. 3, FirstFit routine, with the bitset of Sec. 3.2): colour =
// smallest c > 0 whose bit c-1 is clear in the OR of the neighbours' settled
// colours (X > 0).  Written as FLAG | c.
// ---------------------------------------------------------------------------

// Tile buckets: a wavefront takes 64 worklist entries at a time; L lanes per vertex,
// 64/L vertices per sub-step, L sub-steps.  Degree <= 4L-3 <= 61, so the mex is
// <= 62 and a single 64-bit register mask is exact.
template <int L>
__device__ __forceinline__ void assign_tiles(const RoundArgs& a, const int* list, int lo, int hi,
                                             int* res, long long& arcs) {
    constexpr int V = 64 / L;
    const int lane = __lane_id();
    const int q = lane & (L - 1);
    const int jsub = lane / L;
    int wlo, whi;
    wave_slice(lo, hi, wlo, whi);
    for (int t0 = wlo; t0 < whi; t0 += 64) {
        const int nv = min(64, whi - t0);
        const int i = t0 + lane;
        const int v_l = lane < nv ? list[i] : -1;
        int beg_l = 0, end_l = 0;
        if (v_l >= 0) {
            beg_l = a.rowptr[v_l];
            end_l = a.rowptr[v_l + 1];
        }
        const int nsub = (nv + V - 1) / V;
        for (int sstep = 0; sstep < nsub; ++sstep) {
            const int j = sstep * V + jsub;
            const int beg = __shfl(beg_l, j, 64);
            const int end = __shfl(end_l, j, 64);
            int w[4];
            load_quad(a.colidx, a.nnz, beg, end, q, w);
            int x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = w[k] >= 0 ? a.X[w[k]] : 0;
            unsigned long long m = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (x[k] > 0 && x[k] <= 64) m |= 1ull << (x[k] - 1);
            m = group_or<L>(m);
            if (q == 0) res[j] = __ffsll((long long)~m);
        }
        __builtin_amdgcn_wave_barrier();
        if (v_l >= 0) {
            a.X[v_l] = FLAG | res[lane];
            arcs += end_l - beg_l;
            if (end_l - beg_l > 4 * L - 3) atomicOr(&a.ctl->err, 8);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Lane-per-vertex FirstFit for the tile buckets (degree <= 61): every lane walks its
// own row quad by quad; the mask stays in the lane, no cross-lane reduction.  On
// meshes the k-th neighbours of consecutive vertices are consecutive, so the colour
// gathers of a wavefront coalesce.
__device__ __forceinline__ void assign_lanes(const RoundArgs& a, const int* list, int lo, int hi,
                                             long long& arcs) {
    const int lane = __lane_id();
    int wlo, whi;
    wave_slice(lo, hi, wlo, whi);
    for (int t0 = wlo; t0 < whi; t0 += 64) {
        const int nv = min(64, whi - t0);
        const int v_l = lane < nv ? list[t0 + lane] : -1;
        int beg = 0, end = 0;
        if (v_l >= 0) {
            beg = a.rowptr[v_l];
            end = a.rowptr[v_l + 1];
        }
        const int mis = (int)((reinterpret_cast<uintptr_t>(a.colidx) >> 2) & 3);
        const int nq = end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
        unsigned long long m = 0;
        for (int q = 0; q < nq; ++q) {
            int w[4];
            load_quad(a.colidx, a.nnz, beg, end, q, w);
            int x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = w[k] >= 0 ? a.X[w[k]] : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (x[k] > 0 && x[k] <= 64) m |= 1ull << (x[k] - 1);
        }
        if (v_l >= 0) {
            a.X[v_l] = FLAG | __ffsll((long long)~m);
            arcs += end - beg;
            if (end - beg > 63) atomicOr(&a.ctl->err, 8);
        }
    }
}

// Wavefront bucket (62 .. t_wave <= 1024): metadata for 64 vertices at a time, then
// the whole wavefront scans one row with 16-byte quads; colours 1..64 in a register
// mask, 65..1088 in a per-wavefront LDS bitmap.
__device__ __forceinline__ void assign_wave(const RoundArgs& a, const int* list, int lo, int hi,
                                            unsigned* ovf, int* res, long long& arcs) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    unsigned* my = ovf + wv * OVW;
    int wlo, whi;
    wave_slice(lo, hi, wlo, whi);
    for (int t0 = wlo; t0 < whi; t0 += 64) {
        const int nv = min(64, whi - t0);
        const int v_l = lane < nv ? list[t0 + lane] : -1;
        int beg_l = 0, end_l = 0;
        if (v_l >= 0) {
            beg_l = a.rowptr[v_l];
            end_l = a.rowptr[v_l + 1];
        }
        for (int j = 0; j < nv; ++j) {
            const int beg = __builtin_amdgcn_readlane(beg_l, j);
            const int end = __builtin_amdgcn_readlane(end_l, j);
            if (lane < OVW) my[lane] = 0;
            __builtin_amdgcn_wave_barrier();
            unsigned long long m = 0;
            const int nq = ((end - beg) + 3 + 3) / 4 + 1;     // quads that can overlap the row
            for (int q0 = 0; q0 < nq; q0 += 64) {
                int w[4];
                load_quad(a.colidx, a.nnz, beg, end, q0 + lane, w);
                int x[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) x[k] = w[k] >= 0 ? a.X[w[k]] : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (x[k] > 0) {
                        if (x[k] <= 64) {
                            m |= 1ull << (x[k] - 1);
                        } else {
                            const int kk = x[k] - 65;
                            if (kk < OVW * 32) atomicOr(&my[kk >> 5], 1u << (kk & 31));
                        }
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
            if (lane == 0) res[j] = c;
            __builtin_amdgcn_wave_barrier();
        }
        if (v_l >= 0) {
            a.X[v_l] = FLAG | res[lane];
            arcs += end_l - beg_l;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Smallest colour > base0 absent from the settled neighbours of row [beg, end),
// computed by the whole workgroup over LDS bitmap windows of 32768 colours (a
// further window only if one is completely forbidden).  Every thread must call.
__device__ __forceinline__ int wg_mex_window(const RoundArgs& a, int beg, int end, int base0, RoundLds& s) {
    const int nq = ((end - beg) + 3 + 3) / 4 + 1;
    int base = base0, c = 0;
    for (;;) {
        for (int k = threadIdx.x; k < BMW; k += WG) s.bm[k] = 0;
        __syncthreads();
        for (int q0 = 0; q0 < nq; q0 += WG) {
            int w[4];
            load_quad(a.colidx, a.nnz, beg, end, q0 + (int)threadIdx.x, w);
            int x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = w[k] >= 0 ? a.X[w[k]] : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int kk = x[k] - 1 - base;
                if (x[k] > 0 && (unsigned)kk < (unsigned)(BMW * 32)) atomicOr(&s.bm[kk >> 5], 1u << (kk & 31));
            }
        }
        __syncthreads();
        int best = 0x7fffffff;
        for (int k = threadIdx.x; k < BMW; k += WG) {
            const unsigned wd = s.bm[k];
            if (wd != 0xffffffffu) best = min(best, k * 32 + __ffs(~wd) - 1);
        }
        best = block_min(best, s.red);
        if (best != 0x7fffffff) {
            c = base + best + 1;
            break;
        }
        base += BMW * 32;
    }
    return c;
}

// Workgroup bucket (t_wave .. t_split): one workgroup per vertex, taken dynamically.
__device__ __forceinline__ void assign_wg(const RoundArgs& a, const int* list, int cnt, RoundLds& s,
                                          long long& arcs) {
    for (;;) {
        if (threadIdx.x == 0) s.sh[0] = atomicAdd(&a.ctl->dyn[0][5], 1);
        __syncthreads();
        const int i = s.sh[0];
        __syncthreads();
        if (i >= cnt) break;
        const int v = list[i];
        const int beg = a.rowptr[v], end = a.rowptr[v + 1];
        const int c = wg_mex_window(a, beg, end, 0, s);
        if (threadIdx.x == 0) {
            a.X[v] = FLAG | c;
            arcs += end - beg;
        }
    }
}

// Device-scope atomic access to the split-row merge state.  These are performed at
// the device coherence point, so no L2 writeback / invalidate fence is needed; the
// order "my contributions, then my done-count" is kept by waiting for the returned
// values of the contributions (wait_on) before issuing the count.
__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned or_agent(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_agent(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back (Merrill and Garland's single-pass prefix scan), run by one
// whole wavefront: unit u publishes its count c, then reads the status words of the
// 64 units before it at once and adds up counts back to the nearest unit that has
// published its inclusive prefix (further windows of 64 if none has), and publishes
// its own.  Status words: high half 0 = nothing yet, 1 = count, 2 = inclusive prefix;
// low half the value.  Units are numbered in the order their blocks took a ticket, so
// every unit waited on belongs to a block that is already running and publishes its
// count without waiting: the walk always ends.  Returns the exclusive prefix of u in
// every lane (-1 if the walk gave up; the caller then takes an unordered position).
__device__ __forceinline__ void lookback_publish(unsigned long long* st, int u, int c) {
    if (__lane_id() == 0) st_agent(&st[u], ((u == 0 ? 2ull : 1ull) << 32) | (unsigned)c);
}
__device__ __forceinline__ int lookback_walk(unsigned long long* st, int u, int c, int* err) {
    const int lane = __lane_id();
    if (u == 0) return 0;
    int excl = 0;
    int spins = 0;
    for (int base = u - 1;;) {
        // safety net: a unit that never publishes would be a bug; flag it (the host
        // then fails the call) rather than spin forever
        if (++spins > (1 << 22)) {
            if (lane == 0) atomicOr(err, ERR_LOOKBACK);
            return -1;
        }
        const int k = base - lane;
        const unsigned long long x = k >= 0 ? ld_agent(&st[k]) : (2ull << 32);   // before unit 0: prefix 0
        const unsigned kind = (unsigned)(x >> 32);
        const unsigned long long incl = __ballot(kind == 2);
        const unsigned long long notready = __ballot(kind == 0);
        // the lanes up to the nearest inclusive prefix (or all 64) must have published
        const int stop = incl ? __ffsll((long long)incl) - 1 : 63;
        const unsigned long long need = (2ull << stop) - 1ull;
        if (notready & need) continue;
        int v = lane <= stop ? (int)(unsigned)x : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        excl += v;
        if (incl) break;
        base -= 64;
    }
    if (lane == 0) st_agent(&st[u], (2ull << 32) | (unsigned)(excl + c));
    return excl;
}
__device__ __forceinline__ int lookback(unsigned long long* st, int u, int c, int* err) {
    lookback_publish(st, u, c);
    return lookback_walk(st, u, c, err);
}

// Makes the wavefront wait until `v` (the result of an atomic) has arrived, and keeps
// later memory operations after that point.
__device__ __forceinline__ void wait_on(unsigned v) { asm volatile("" ::"v"(v) : "memory"); }

// Split bucket (> t_split): the row of a queued hub is cut into SPLIT_CH-arc chunks,
// one workgroup per chunk (chunk t belongs to queue entry owner[t]).  Each chunk ORs
// the colours it sees (1..32*HW) into the hub's bitmap with device atomics, then
// counts itself done; the chunk that completes the count picks the colour.  If all
// colours 1..32*HW are forbidden it rescans the whole row for higher ones.
__device__ __forceinline__ void assign_split(const RoundArgs& a, const int* list, int nchunks, int j, int nbk,
                                             RoundLds& s, long long& arcs) {
    const int* cstart = a.cstart[a.par_in];
    const int* owner = a.owner[a.par_in];
    const int tid = threadIdx.x;
    for (int t = j; t < nchunks; t += nbk) {
        const int p = owner[t];
        const int v = list[p];
        const int k = t - cstart[p];
        const int rb = a.rowptr[v], re = a.rowptr[v + 1];
        const int nch = split_chunks(re - rb);
        const int beg = rb + k * SPLIT_CH, end = min(beg + SPLIT_CH, re);
        if (tid < HW) s.bm[tid] = 0;
        __syncthreads();
        const int nq = ((end - beg) + 3 + 3) / 4 + 1;
        for (int q0 = 0; q0 < nq; q0 += WG) {
            int w[4];
            load_quad(a.colidx, a.nnz, beg, end, q0 + tid, w);
            int x[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) x[kk] = w[kk] >= 0 ? a.X[w[kk]] : 0;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int cb = x[kk] - 1;
                if (x[kk] > 0 && cb < HW * 32) atomicOr(&s.bm[cb >> 5], 1u << (cb & 31));
            }
        }
        __syncthreads();
        if (tid < 64) {
            // wavefront 0 publishes the chunk's colours, waits for the atomics to be
            // performed, then counts the chunk done
            unsigned old = 0;
            if (tid < HW) {
                const unsigned wd = s.bm[tid];
                if (wd) old = or_agent(&a.hubbm[p * HW + tid], wd);
            }
            wait_on(old);
            __builtin_amdgcn_wave_barrier();
            if (tid == 0) s.sh[1] = add_agent(&a.hubdone[p], 1) == nch - 1;
        }
        __syncthreads();
        if (s.sh[1]) {
            const unsigned wd = tid < HW ? ld_agent(&a.hubbm[p * HW + tid]) : 0xffffffffu;
            int best = wd != 0xffffffffu ? tid * 32 + __ffs(~wd) - 1 : 0x7fffffff;
            best = block_min(best, s.red);
            const int c = best != 0x7fffffff ? best + 1 : wg_mex_window(a, rb, re, HW * 32, s);
            if (tid < HW) st_agent(&a.hubbm[p * HW + tid], 0u);
            if (tid == 0) {
                st_agent(&a.hubdone[p], 0);
                a.X[v] = FLAG | c;
                arcs += re - rb;
            }
        }
        __syncthreads();
    }
}

// One FirstFit phase for the block `bid` of a grid partitioned by boff.
__device__ __forceinline__ void assign_phase(const RoundArgs& a, RoundLds& s, int bid, const int* boff) {
    int b, j, nbk;
    block_bucket(boff, bid, b, j, nbk);
    if (bid == 0 && threadIdx.x == 0) {
        for (int k = 0; k < NB; ++k) {
            a.ctl->cnt[a.par_out][k] = 0;
            a.ctl->dyn[1][k] = 0;
            st_agent(&a.ctl->tk[k], 0);
        }
        a.ctl->ccnt[a.par_out] = 0;
        a.ctl->nsettled = 0;
        a.ctl->pround += 1;
    }
    // the conflict test of this round uses one look-back status word per block of its
    // grid (the FirstFit grid may be smaller)
    if (a.lbs && threadIdx.x == 0)
        for (int i = bid; i < a.lbs_n; i += gridDim.x) st_agent(&a.lbs[i], 0ull);
    if (bid >= boff[NB]) return;
    const int cnt = a.ctl->cnt[a.par_in][b];
    const int* list = a.wl_in + a.seg[b];
    const int lo = (int)((long long)j * cnt / nbk);
    const int hi = (int)((long long)(j + 1) * cnt / nbk);
    int* res = s.res + (threadIdx.x >> 6) * 64;
    long long arcs = 0;
    if (a.pushff) {
        // every bucket, split hubs included, is one lane per vertex in push mode
        assign_push(a, list, lo, hi, arcs);
    } else if (b < NTILE && (a.lane_mode_assign >> b & 1)) {
        assign_lanes(a, list, lo, hi, arcs);
    } else {
        switch (b) {
            case 0: assign_tiles<2>(a, list, lo, hi, res, arcs); break;
            case 1: assign_tiles<4>(a, list, lo, hi, res, arcs); break;
            case 2: assign_tiles<8>(a, list, lo, hi, res, arcs); break;
            case 3: assign_tiles<16>(a, list, lo, hi, res, arcs); break;
            case 4: assign_wave(a, list, lo, hi, s.ovf, res, arcs); break;
            case 5: assign_wg(a, list, cnt, s, arcs); break;
            default: assign_split(a, list, a.ctl->ccnt[a.par_in], j, nbk, s, arcs); break;
        }
    }
    if (a.st_arcs) {
        // 0-based index of this round: the rounds completed so far (stable during FirstFit)
        const int ridx = ld_agent(&a.ctl->rounds);
        const long long t = block_sum64(arcs, s.red64);
        if (threadIdx.x == 0 && t && ridx < a.st_cap)
            atomicAdd((unsigned long long*)&a.st_arcs[ridx], (unsigned long long)t);
    }
}

// Queue sizes of the round that reads parity `par` (the split bucket counted in chunks).
__device__ __forceinline__ void queue_sizes(const Ctl* ctl, int par, int* cnt) {
    for (int b = 0; b < NB; ++b) cnt[b] = ctl->cnt[par][b];
    cnt[BSPLIT] = ctl->ccnt[par];
}

__global__ __launch_bounds__(WG) void k_assign(RoundArgs a) {
    __shared__ RoundLds s;
    __shared__ int boff[NB + 1];
    if (threadIdx.x == 0) {
        if (a.dev_plan) {
            int cnt[NB];
            queue_sizes(a.ctl, a.par_in, cnt);
            device_plan(cnt, gridDim.x, boff, 1);
        } else {
            for (int k = 0; k <= NB; ++k) boff[k] = a.boff[k];
        }
    }
    __syncthreads();
    assign_phase(a, s, blockIdx.x, boff);
}

// ---------------------------------------------------------------------------
// Conflict test (Sec. 3, ConflictResolve, requeue direction fixed to the higher
// id) + colour clearing + worklist push by prefix sums (Sec. 3.1).  A vertex loses
// iff some neighbour w < v holds the same tentative colour.  Winners write their
// final colour and the 0-based output; a loser's X keeps the FLAG (uncoloured for
// the next FirstFit) and its id goes to the next worklist.
// ---------------------------------------------------------------------------

template <bool W>
__device__ __forceinline__ void settle(const RoundArgs& a, int v, int cv, int& cmax) {
    a.X[v] = cv;
    a.out[v] = cv - 1;
    if (W) a.srnd[v] = wround_of(a);       // wake flags: the settling round, for the statistics
    cmax = max(cmax, cv);
}

// Writes the per-wavefront loser buffers to the global worklist with one atomic per
// workgroup; in ordered mode (unit_st) at the position a look-back gives, so the
// worklist keeps ascending id order from round to round.  `wc` is the calling wavefront's count (uniform).  Buffers hold
// ascending worklist positions and wavefronts own ascending slices, so each flush
// is one run in worklist order.
__device__ __forceinline__ void flush_losers(RoundLds& s, int wc, int* outl, int* cnt_out,
                                             unsigned long long* unit_st, int unit, int* err) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    if (lane == 0) s.wcnt[wv] = wc;
    __syncthreads();
    int lbase = 0;
    if (unit_st && wv == 0) {
        // ordered: this block's run goes right after the runs of the blocks before it
        int tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += s.wcnt[w];
        lbase = lookback(unit_st, unit, tot, err);
    }
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += s.wcnt[w];
        int base;
        if (unit_st && lbase >= 0) {
            base = lbase;
            if (tot) atomicAdd(cnt_out, tot);
        } else {
            base = tot ? atomicAdd(cnt_out, tot) : 0;
        }
        for (int w = 0; w < WAVES; ++w) {
            s.wbase[w] = base;
            base += s.wcnt[w];
        }
    }
    __syncthreads();
    const int* src = s.lbuf + wv * WAVE_CAP;
    int* dst = outl + s.wbase[wv];
    for (int k = lane; k < wc; k += 64) dst[k] = src[k];
    __syncthreads();
}

// Appends the losers among this wavefront's 64 tile entries (one per lane) to the
// wavefront buffer in lane order.
__device__ __forceinline__ void push_losers(int v_l, bool lost_l, int* mybuf, int& wc) {
    const unsigned long long lm = __ballot(v_l >= 0 && lost_l);
    if (v_l >= 0 && lost_l) mybuf[wc + __popcll(lm & lanemask_lt())] = v_l;
    wc += __popcll(lm);
}

template <int L, bool W>
__device__ __forceinline__ void detect_tiles(const RoundArgs& a, const int* list, int lo, int hi, RoundLds& s,
                                             int* outl, int* cnt_out, int& cmax, unsigned long long* ust, int unit) {
    constexpr int V = 64 / L;
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int q = lane & (L - 1);
    const int jsub = lane / L;
    const unsigned long long gmask = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
    const int gshift = lane & ~(L - 1);
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wlo, whi;
        wave_slice(s0, s1, wlo, whi);      // <= WAVE_CAP entries per wavefront
        int wc = 0;
        // two 64-entry batches per step (entry u * 64 + lane), each stage's loads for
        // both issued together so their latencies overlap
        int* ids = s.idx + wv * 128;
        int* res2 = s.res2 + wv * 128;
        for (int t0 = wlo; t0 < whi; t0 += 128) {
            int v_l[2], beg_l[2] = {0, 0}, end_l[2] = {0, 0}, cv_l[2] = {0, 0}, h_l[2] = {-1, -1};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + 64 * u + lane;
                v_l[u] = t < whi ? list[t] : -1;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (v_l[u] >= 0) {
                    cv_l[u] = tentative(a, v_l[u]);
                    if (a.hint) h_l[u] = a.hint[v_l[u]];
                }
            }
            bool hinted_l[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                // the remembered neighbour still requeues v (see hint_hit)
                const int h = h_l[u];
                hinted_l[u] = h >= 0 && (a.rule != 0 || h < v_l[u]) && (a.X[h] & CMASK) == cv_l[u];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (v_l[u] >= 0 && !hinted_l[u]) {
                    beg_l[u] = a.rowptr[v_l[u]];
                    end_l[u] = a.rowptr[v_l[u] + 1];
                }
            }
            // only the vertices the hint did not decide are tested: their entries are
            // listed in ids, V of them per sub-step
            const unsigned long long todo0 = __ballot(v_l[0] >= 0 && !hinted_l[0]);
            const unsigned long long todo1 = __ballot(v_l[1] >= 0 && !hinted_l[1]);
            const int nt0 = __popcll(todo0);
            const int nt = nt0 + __popcll(todo1);
            res2[lane] = 0;
            res2[64 + lane] = 0;
            if (todo0 >> lane & 1) ids[__popcll(todo0 & lanemask_lt())] = lane;
            if (todo1 >> lane & 1) ids[nt0 + __popcll(todo1 & lanemask_lt())] = 64 + lane;
            __builtin_amdgcn_wave_barrier();
            const int nsub = (nt + V - 1) / V;
            for (int sstep = 0; sstep < nsub; ++sstep) {
                const int jj = sstep * V + jsub;
                const bool real = jj < nt;
                const int e = real ? ids[jj] : lane;      // spare groups repeat their own lane, idle
                const int l = e & 63;
                const bool hi1 = e >= 64;
                // every lane takes part in the cross-lane reads (a read from a lane that
                // skipped the instruction would return 0); spare groups then idle
                const int va = __shfl(v_l[0], l, 64), vb = __shfl(v_l[1], l, 64);
                const int ba = __shfl(beg_l[0], l, 64), bb = __shfl(beg_l[1], l, 64);
                const int ea = __shfl(end_l[0], l, 64), eb = __shfl(end_l[1], l, 64);
                const int ca = __shfl(cv_l[0], l, 64), cb = __shfl(cv_l[1], l, 64);
                const int v = hi1 ? vb : va;
                const int cv = hi1 ? cb : ca;
                int beg = hi1 ? bb : ba;
                int end = hi1 ? eb : ea;
                if (!real) beg = end = 0;
                int w[4];
                load_quad(a.colidx, a.nnz, beg, end, q, w);
                int found = -1;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (loses_to(a, w[k], v, cv, end - beg)) found = w[k];
                if (found >= 0 && a.hint) a.hint[v] = found | (W ? a.hflag : 0);    // any conflicting neighbour will do
                const bool lost = ((__ballot(found >= 0) >> gshift) & gmask) != 0;
                if (q == 0 && real) res2[e] = lost;
            }
            __builtin_amdgcn_wave_barrier();
            bool lost_l[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) lost_l[u] = hinted_l[u] || res2[64 * u + lane] != 0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (v_l[u] >= 0 && !lost_l[u]) settle<W>(a, v_l[u], cv_l[u], cmax);
                if (a.pushff) push_rows_wave<W>(a, v_l[u] >= 0 && !lost_l[u], v_l[u], cv_l[u], beg_l[u], end_l[u]);
                push_losers(v_l[u], lost_l[u], mybuf, wc);
            }
        }
        flush_losers(s, wc, outl, cnt_out, ust, unit, &a.ctl->err);
    }
}

// Lane-per-vertex conflict test for the tile buckets: every lane walks the lower part
// of its own row quad by quad and stops at its first conflict (or, for sorted rows,
// at its first w >= v); the wavefront moves on when all its lanes have stopped.
template <bool W>
__device__ __forceinline__ void detect_lanes(const RoundArgs& a, const int* list, int lo, int hi, RoundLds& s,
                                             int* outl, int* cnt_out, int& cmax, unsigned long long* ust, int unit) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    const int mis = (int)((reinterpret_cast<uintptr_t>(a.colidx) >> 2) & 3);
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wlo, whi;
        wave_slice(s0, s1, wlo, whi);
        int wc = 0;
        for (int t0 = wlo; t0 < whi; t0 += 64) {
            const int nv = min(64, whi - t0);
            const int v_l = lane < nv ? list[t0 + lane] : -1;
            int beg = 0, end = 0, cv = 0;
            bool lost = false;
            if (v_l >= 0) {
                cv = tentative(a, v_l);
                lost = hint_hit(a, v_l, cv);
                if (!lost) {
                    beg = a.rowptr[v_l];
                    end = a.rowptr[v_l + 1];
                }
            }
            const int nq = end > beg ? (((end - 1 + mis) >> 2) - ((beg + mis) >> 2) + 1) : 0;
            int found = -1;
            for (int q = 0; q < nq; ++q) {
                int w[4];
                load_quad(a.colidx, a.nnz, beg, end, q, w);
                bool stop = false;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (w[k] >= 0) {
                        if (a.rule == 0 && w[k] >= v_l) {
                            stop |= a.sorted != 0;
                        } else if (found < 0 && loses_to(a, w[k], v_l, cv, end - beg)) {
                            found = w[k];
                        }
                    }
                }
                if (found >= 0 || stop) break;
            }
            if (found >= 0) {
                lost = true;
                if (a.hint) a.hint[v_l] = found | (W ? a.hflag : 0);
            }
            if (v_l >= 0 && !lost) settle<W>(a, v_l, cv, cmax);
            if (a.pushff) push_rows_wave<W>(a, v_l >= 0 && !lost, v_l, cv, beg, end);
            push_losers(v_l, lost, mybuf, wc);
        }
        flush_losers(s, wc, outl, cnt_out, ust, unit, &a.ctl->err);
    }
}

// ---------------------------------------------------------------------------
// Live lists (id rule), built lazily.  A vertex of degree > 61 may stay on the
// worklist for many rounds, and most of its lower neighbours settle early; once
// settled, a neighbour can never conflict with it again (FirstFit excluded its
// colour).  So each test of such a vertex keeps the lower neighbours it finds still
// uncoloured in a live list (same offsets as its row, in a separate array): a test
// scans the list first, dropping the entries it finds settled (packed to the front as
// it goes), and then the row entries no test has examined yet, from a resume
// position, appending the lower uncoloured ones.  Every scan stops at the step that
// finds a conflict: when the list part stops early, the gap left in its scanned part
// is filled from the end of the list, so the list stays contiguous and its unscanned
// entries are kept; when the row part stops early, the resume position marks the
// first entry not examined.  Entries are tested before they are dropped, so a
// neighbour settling in this very round is still compared.  A split row keeps a
// list and a resume position per chunk.
// ---------------------------------------------------------------------------

// Whether row entry w beats v (degree dv) under the round's rule: a lower id (id rule),
// or a larger degree, the lower id on equal degree (degree rule).
__device__ __forceinline__ bool beats_v(const RoundArgs& a, int w, int v, int dv) {
    return w != v && beats(a.rule, a.rowptr, w, v, dv);
}

// Scan step: reads the entries of src[beg, end) in quad q of the range, tests them
// against v (degree dv) and returns the neighbours that beat v and are still
// uncoloured in keep/w.  `row`: the entries come from v's row (under the id rule, for
// sorted rows an entry >= v ends the lower part); list entries beat v already.
__device__ __forceinline__ void live_step(const RoundArgs& a, const int* src, int beg, int end, int q, int v,
                                          int dv, int cv, bool row, int w[4], unsigned& keep, bool& hit,
                                          bool& stop, int hf) {
    load_quad(src, a.nnz, beg, end, q, w);
    keep = 0;
    int found = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (w[k] < 0) continue;
        if (!row || beats_v(a, w[k], v, dv)) {
            const int x = a.X[w[k]];
            if ((x & CMASK) == cv) found = w[k];
            if (x <= 0) keep |= 1u << k;
        } else {
            stop |= a.rule == 0 && w[k] >= v && a.sorted;   // sorted rows: no lower entries further on
        }
    }
    if (found >= 0) {
        hit = true;
        if (a.hint) a.hint[v] = found | hf;     // any conflicting neighbour will do
    }
}

// The whole wavefront runs the conflict test of v (tentative colour cv, degree dv)
// over the range [rb, re) of its row (the whole row, or a chunk of a split row): its
// live list live[rb, rb + len), then the unexamined entries colidx[p, re) (len < 0:
// nothing examined yet, i.e. len = 0 and p = rb).  Stores the new length and resume
// position at *lenp and *posp; returns whether a conflict was found.  Every lane must
// call.
__device__ __forceinline__ bool live_test_wave(const RoundArgs& a, int v, int dv, int cv, int rb, int re, int len,
                                               int p, int* lenp, int* posp, int hf) {
    const int lane = __lane_id();
    if (len < 0) {
        len = 0;
        p = rb;
    }
    int K = 0;                 // entries kept so far, packed at live[rb ...]
    bool lost = false;
    if (len > 0) {
        const int send = rb + len;
        const int nq = quad_count(a.live, rb, send);
        int scanned = len;     // list positions scanned
        for (int q0 = 0; q0 < nq; q0 += 64) {
            int w[4];
            unsigned keep;
            bool hit = false, stop = false;
            live_step(a, a.live, rb, send, q0 + lane, v, dv, cv, false, w, keep, hit, stop, hf);
            int tot;
            int pos = rb + K + wave_excl(__popc(keep), tot);
            const int qs = rb + quad_end(a.live, rb, q0 + lane);   // position of w[0]
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (keep >> k & 1) {
                    if (pos != qs + k) a.live[pos] = w[k];   // an entry already in place stays
                    ++pos;
                }
            }
            K += tot;
            if (__ballot(hit) != 0) {
                lost = true;
                scanned = min(len, quad_end(a.live, rb, q0 + 64));
                break;
            }
        }
        // fill the gap [K, scanned) from the end of the unscanned part [scanned, len)
        const int m = min(scanned - K, len - scanned);
        for (int i = lane; i < m; i += 64) a.live[rb + K + i] = a.live[rb + len - m + i];
        K = len - (scanned - K);
    }
    if (!lost && p < re) {
        const int nq = quad_count(a.colidx, p, re);
        int np = re;           // resume position after this scan
        for (int q0 = 0; q0 < nq; q0 += 64) {
            int w[4];
            unsigned keep;
            bool hit = false, stop = false;
            live_step(a, a.colidx, p, re, q0 + lane, v, dv, cv, true, w, keep, hit, stop, hf);
            int tot;
            int pos = rb + K + wave_excl(__popc(keep), tot);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (keep >> k & 1) a.live[pos++] = w[k];
            }
            K += tot;
            const bool anyhit = __ballot(hit) != 0;
            lost |= anyhit;
            if (__ballot(stop) != 0) break;       // sorted: the lower part is complete
            if (anyhit) {
                np = min(re, p + quad_end(a.colidx, p, q0 + 64));
                break;
            }
        }
        p = np;
    }
    if (lane == 0) {
        *lenp = K;
        *posp = p;
    }
    return lost;
}

// Lane-parallel first look at a live-list test (every lane its own vertex or chunk):
// the first quad of the list, or of the unexamined row entries when the list is
// empty.  Reads only.  Returns 1 if that quad holds a conflicting neighbour, -1 if
// nothing is left to examine (no lower uncoloured neighbour remains: no conflict), 0
// otherwise (the full test decides).
__device__ __forceinline__ int live_probe(const RoundArgs& a, int v, int dv, int cv, int rb, int re, int len,
                                          int p, int hf) {
    if (len < 0) {
        len = 0;
        p = rb;
    }
    if (len == 0 && p >= re) return -1;
    int w[4];
    if (len > 0) load_quad(a.live, a.nnz, rb, rb + len, 0, w);
    else load_quad(a.colidx, a.nnz, p, re, 0, w);
    int found = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (w[k] >= 0 && (len > 0 || beats_v(a, w[k], v, dv)) && (a.X[w[k]] & CMASK) == cv) found = w[k];
    if (found < 0) return 0;
    if (a.hint) a.hint[v] = found | hf;
    return 1;
}

// Lane-streamed conflict test (id rule, unordered compaction).  Every lane runs its
// own vertex through the steps of the test and takes the next worklist entry as soon
// as that vertex is decided, so the wavefront keeps 64 independent chains of
// dependent loads in flight instead of waiting for its slowest vertex.  A loop pass
// waits once for the loads the previous pass issued, advances every lane by one step
// and issues the loads of its next step:
//   meta:   the vertex's colour word, hint and row bounds (LONG: and its live-list
//           length and resume position), and the lane's next worklist entry
//   hint:   the hint's colour word and the first quad to examine
//   gather: the colour words of the quad's lower entries, and the next quad
// The quads examined are the row's (rows of at most 61 arcs) or, with LONG (rows with
// live lists), the live list's and then the unexamined row entries' (see the live
// lists below); this walk only reads.  A vertex loses at a hint that still conflicts
// (see hint_hit) or at the first lower neighbour holding its tentative colour, and
// wins when nothing is left to examine (sorted rows: no lower entry).  A LONG vertex
// still undecided after DEFER_QUADS quads is deferred: after the stream the wavefront
// tests the deferred ones together (live_test_wave, which also updates their lists).
// Winners are staged per wavefront and push their rows 64 at a time; losers go to the
// wavefront's buffer in the order they are decided, deferred vertices to its other end.
constexpr int DEFER_QUADS = 16;

template <bool W, bool LONG>
__device__ __forceinline__ void detect_stream(const RoundArgs& a, const int* list, int lo, int hi, RoundLds& s,
                                              int* outl, int* cnt_out, int& cmax, unsigned long long* ust, int unit) {
    constexpr int S_IDLE = 0, S_META = 1, S_HINT = 2, S_GATHER = 3;
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    int* wb = s.wbuf + wv * (4 * 128);
    const int hf = W ? a.hflag : 0;
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wlo, whi;
        wave_slice(s0, s1, wlo, whi);
        int wc = 0;               // losers at mybuf[0 .. wc)
        int nd = 0;               // deferred vertices at mybuf[WAVE_CAP - nd .. WAVE_CAP)
        int nwin = 0;             // winners staged in wb
        int next = wlo + 64;      // first worklist entry no lane has claimed
        int vn = wlo + lane < whi ? list[wlo + lane] : -1;   // the lane's next vertex
        int st = S_IDLE;
        bool fresh = true;        // first pass: every lane with an entry starts it
        int v = -1, cv = 0, h = -1, beg = 0, end = 0;
        int len = 0, p = 0;       // LONG: list length and resume position
        int seg = 1, qi = 0, nqL = 0, nqR = 0, walked = 0;
        int cur[4] = {-1, -1, -1, -1}, nxt[4] = {-1, -1, -1, -1};
        int rX = 0, rH = -1, rB = 0, rE = 0, rL = -1, rP = 0, rHX = 0;
        int rG[4] = {0, 0, 0, 0};
        for (;;) {
            // consume the loads of the previous pass and take one step
            bool lose = false, win = false, defer = false, doHint = false, doQuad = false, doGather = false;
            int qseg = 1, qload = 0;  // the quad to load: segment (0 list, 1 row) and index
            if (st == S_META) {
                cv = rX & CMASK;
                beg = rB;
                end = rE;
                h = (rH != -1 && (rH & IDMASK) < v) ? (rH & IDMASK) : -1;
                len = 0;
                p = beg;
                if (LONG && rL >= 0) {
                    len = rL;
                    p = rP;
                }
                nqL = LONG ? quad_count(a.live, beg, beg + len) : 0;
                nqR = quad_count(a.colidx, p, end);
                walked = 0;
                if (nqL + nqR == 0) {
                    win = true;
                } else {
                    seg = nqL > 0 ? 0 : 1;
                    qi = 0;
                    doHint = h >= 0;
                    doQuad = true;
                    qseg = seg;
                    qload = 0;
                    st = S_HINT;
                }
            } else if (st == S_HINT || st == S_GATHER) {
                bool stop = false;
                if (st == S_HINT) {
                    lose = h >= 0 && (rHX & CMASK) == cv;
                } else {
                    int found = -1;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (cur[k] >= 0) {
                            if (cur[k] < v) {
                                if ((rG[k] & CMASK) == cv) found = cur[k];
                            } else {
                                stop |= seg == 1 && a.sorted != 0;   // sorted rows: no lower entries further on
                            }
                        }
                    }
                    if (found >= 0) {
                        lose = true;
                        if (a.hint) a.hint[v] = found | hf;     // any conflicting neighbour will do
                    }
                    ++walked;
                }
                if (!lose) {
                    // the quad to examine next: the one loaded last pass (at S_HINT: the first)
                    int ns = seg, nqi = qi;
                    bool have = true;
                    if (st == S_GATHER) {
                        if (stop) {
                            have = false;
                        } else if (seg == 0 && qi + 1 < nqL) {
                            nqi = qi + 1;
                        } else if (seg == 0 && nqR > 0) {
                            ns = 1;
                            nqi = 0;
                        } else if (seg == 1 && qi + 1 < nqR) {
                            nqi = qi + 1;
                        } else {
                            have = false;
                        }
                    }
                    if (!have) {
                        win = true;
                    } else if (LONG && walked >= DEFER_QUADS) {
                        defer = true;
                    } else {
                        seg = ns;
                        qi = nqi;
#pragma unroll
                        for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
                        doGather = true;
                        // and the quad after it
                        if (seg == 0 && qi + 1 < nqL) {
                            doQuad = true;
                            qseg = 0;
                            qload = qi + 1;
                        } else if (seg == 0 && nqR > 0) {
                            doQuad = true;
                            qseg = 1;
                            qload = 0;
                        } else if (seg == 1 && qi + 1 < nqR) {
                            doQuad = true;
                            qseg = 1;
                            qload = qi + 1;
                        }
                        st = S_GATHER;
                    }
                }
            }
            if (win) settle<W>(a, v, cv, cmax);
            const unsigned long long lm = __ballot(lose);
            if (lose) mybuf[wc + __popcll(lm & lanemask_lt())] = v;
            wc += __popcll(lm);
            if (LONG) {
                const unsigned long long dm = __ballot(defer);
                if (defer) mybuf[WAVE_CAP - 1 - nd - __popcll(dm & lanemask_lt())] = v;
                nd += __popcll(dm);
            }
            if (a.pushff) {
                const unsigned long long wm = __ballot(win);
                if (win) {
                    const int q = 4 * (nwin + __popcll(wm & lanemask_lt()));
                    wb[q] = v;
                    wb[q + 1] = cv;
                    wb[q + 2] = beg;
                    wb[q + 3] = end;
                }
                nwin += __popcll(wm);
                if (nwin >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    push_rows_wave<W>(a, true, wb[4 * lane], wb[4 * lane + 1], wb[4 * lane + 2], wb[4 * lane + 3]);
                    const int rest = nwin - 64;
                    int t[4] = {0, 0, 0, 0};
                    if (lane < rest) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) t[k] = wb[4 * (64 + lane) + k];
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (lane < rest) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) wb[4 * lane + k] = t[k];
                    }
                    __builtin_amdgcn_wave_barrier();
                    nwin = rest;
                }
            }
            // a decided lane (or, in the first pass, every lane) starts its next vertex
            const bool take = (win || lose || defer || (fresh && st == S_IDLE)) && vn >= 0;
            if (win || lose || defer) st = S_IDLE;
            fresh = false;
            bool doMeta = false;
            if (take) {
                v = vn;
                st = S_META;
                doMeta = true;
            }
            const unsigned long long cm = __ballot(take);
            const int tn = next + __popcll(cm & lanemask_lt());
            next += __popcll(cm);
            if (__ballot(st != S_IDLE) == 0) break;
            // issue the loads of the next step
            if (take) vn = tn < whi ? list[tn] : -1;
            if (doMeta) {
                rX = a.X[v];
                rH = a.hint ? a.hint[v] : -1;
                rB = a.rowptr[v];
                rE = a.rowptr[v + 1];
                if (LONG) {
                    rL = a.llen[v];
                    rP = a.lpos[v];
                }
            }
            if (doHint) rHX = a.X[h];
            if (doQuad) {
                if (LONG && qseg == 0) load_quad(a.live, a.nnz, beg, beg + len, qload, nxt);
                else load_quad(a.colidx, a.nnz, p, end, qload, nxt);
            }
            if (doGather) {
#pragma unroll
                for (int k = 0; k < 4; ++k) rG[k] = (cur[k] >= 0 && cur[k] < v) ? a.X[cur[k]] : 0;
            }
        }
        if (a.pushff && nwin > 0) {
            __builtin_amdgcn_wave_barrier();
            const bool on = lane < nwin;
            push_rows_wave<W>(a, on, on ? wb[4 * lane] : 0, on ? wb[4 * lane + 1] : 0, on ? wb[4 * lane + 2] : 0,
                              on ? wb[4 * lane + 3] : 0);
        }
        if (LONG) {
            // the deferred vertices, 64 at a time: the whole wavefront tests one after
            // another (updating their lists), then winners push and losers are listed
            for (int d0 = 0; d0 < nd; d0 += 64) {
                const bool on = d0 + lane < nd;
                __builtin_amdgcn_wave_barrier();
                const int vd = on ? mybuf[WAVE_CAP - 1 - d0 - lane] : -1;
                __builtin_amdgcn_wave_barrier();
                int bd = 0, ed = 0, cd = 0, ld = -1, pd = 0;
                if (on) {
                    cd = a.X[vd] & CMASK;
                    bd = a.rowptr[vd];
                    ed = a.rowptr[vd + 1];
                    ld = a.llen[vd];
                    pd = a.lpos[vd];
                }
                bool lost_l = false;
                unsigned long long todo = __ballot(on);
                while (todo) {
                    const int j = __ffsll((long long)todo) - 1;
                    todo &= todo - 1;
                    const int vj = __builtin_amdgcn_readlane(vd, j);
                    const bool l = live_test_wave(a, vj, __builtin_amdgcn_readlane(ed, j) - __builtin_amdgcn_readlane(bd, j),
                                                  __builtin_amdgcn_readlane(cd, j), __builtin_amdgcn_readlane(bd, j),
                                                  __builtin_amdgcn_readlane(ed, j), __builtin_amdgcn_readlane(ld, j),
                                                  __builtin_amdgcn_readlane(pd, j), &a.llen[vj], &a.lpos[vj], hf);
                    if (lane == j) lost_l = l;
                }
                if (on && !lost_l) settle<W>(a, vd, cd, cmax);
                if (a.pushff) push_rows_wave<W>(a, on && !lost_l, vd, cd, bd, ed);
                push_losers(vd, on && lost_l, mybuf, wc);
            }
        }
        flush_losers(s, wc, outl, cnt_out, ust, unit, &a.ctl->err);
    }
}

// Wavefront bucket: metadata for 64 vertices at a time, then the wavefront scans the
// lower part of one row at a time (256 arcs per step; for sorted rows the scan stops
// at the first w >= v, and at the first conflict in any case).
template <bool W>
__device__ __forceinline__ void detect_wave(const RoundArgs& a, const int* list, int lo, int hi, RoundLds& s,
                                            int* outl, int* cnt_out, int& cmax, unsigned long long* ust, int unit) {
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    int* mybuf = s.lbuf + wv * WAVE_CAP;
    for (int s0 = lo; s0 < hi; s0 += SUB) {
        const int s1 = min(s0 + SUB, hi);
        int wlo, whi;
        wave_slice(s0, s1, wlo, whi);
        int wc = 0;
        for (int t0 = wlo; t0 < whi; t0 += 64) {
            const int nv = min(64, whi - t0);
            const int v_l = lane < nv ? list[t0 + lane] : -1;
            int beg_l = 0, end_l = 0, cv_l = 0, len_l = -1, pos_l = 0;
            bool lost_l = false, done_l = v_l < 0;
            if (v_l >= 0) {
                cv_l = tentative(a, v_l);
                lost_l = hint_hit(a, v_l, cv_l);
                beg_l = a.rowptr[v_l];
                end_l = a.rowptr[v_l + 1];
                if (a.live && !lost_l) {
                    len_l = a.llen[v_l];
                    pos_l = len_l >= 0 ? a.lpos[v_l] : beg_l;
                }
            }
            if (a.live && v_l >= 0 && !lost_l) {
                // every lane looks at the first quad of its own vertex's list (or unexamined
                // row): most tests end there, the rest get the whole wavefront below
                const int pr = live_probe(a, v_l, end_l - beg_l, cv_l, beg_l, end_l, len_l, pos_l, W ? a.hflag : 0);
                lost_l = pr > 0;
                done_l = pr != 0;
            }
            done_l = done_l || lost_l;
            unsigned long long todo = __ballot(!done_l);
            while (todo) {
                const int j = __ffsll((long long)todo) - 1;
                todo &= todo - 1;
                const int v = __builtin_amdgcn_readlane(v_l, j);
                const int beg = __builtin_amdgcn_readlane(beg_l, j);
                const int end = __builtin_amdgcn_readlane(end_l, j);
                const int cv = __builtin_amdgcn_readlane(cv_l, j);
                if (a.live) {
                    const bool lost = live_test_wave(a, v, end - beg, cv, beg, end, __builtin_amdgcn_readlane(len_l, j),
                                                     __builtin_amdgcn_readlane(pos_l, j), &a.llen[v], &a.lpos[v],
                                                     W ? a.hflag : 0);
                    if (lane == j) lost_l = lost;
                    continue;
                }
                const int nq = ((end - beg) + 3 + 3) / 4 + 1;
                bool lost = false;
                for (int q0 = 0; q0 < nq; q0 += 64) {
                    int w[4];
                    load_quad(a.colidx, a.nnz, beg, end, q0 + lane, w);
                    int found = -1;
                    bool stop = false;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (loses_to(a, w[k], v, cv, end - beg)) found = w[k];
                        stop |= a.sorted && a.rule == 0 && w[k] >= v;
                    }
                    if (found >= 0 && a.hint) a.hint[v] = found | (W ? a.hflag : 0);   // any conflicting neighbour will do
                    if (__ballot(found >= 0)) {
                        lost = true;
                        break;
                    }
                    if (__ballot(stop)) break;
                }
                if (lane == j) lost_l = lost;
            }
            if (v_l >= 0 && !lost_l) settle<W>(a, v_l, cv_l, cmax);
            if (a.pushff) push_rows_wave<W>(a, v_l >= 0 && !lost_l, v_l, cv_l, beg_l, end_l);
            push_losers(v_l, lost_l, mybuf, wc);
        }
        flush_losers(s, wc, outl, cnt_out, ust, unit, &a.ctl->err);
    }
}

template <bool W>
__device__ __forceinline__ void detect_wg(const RoundArgs& a, const int* list, int cnt, RoundLds& s,
                                          int* outl, int* cnt_out, int& cmax) {
    for (;;) {
        // thread 0 takes the next vertex and evaluates its hint once, so every thread of
        // the block sees the same verdict (the scan below may rewrite the hint)
        if (threadIdx.x == 0) {
            const int i0 = atomicAdd(&a.ctl->dyn[1][5], 1);
            s.sh[0] = i0;
            s.sh[1] = i0 < cnt ? (int)hint_hit(a, list[i0], tentative(a, list[i0])) : 0;
        }
        __syncthreads();
        const int i = s.sh[0];
        bool lost = s.sh[1] != 0;
        __syncthreads();
        if (i >= cnt) break;
        const int v = list[i];
        const int beg = a.rowptr[v], end = a.rowptr[v + 1];
        const int cv = tentative(a, v);
        const int nq = lost ? 0 : ((end - beg) + 3 + 3) / 4 + 1;
        for (int q0 = 0; q0 < nq; q0 += WG) {
            int w[4];
            load_quad(a.colidx, a.nnz, beg, end, q0 + (int)threadIdx.x, w);
            bool hit = false, stop = false;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (loses_to(a, w[k], v, cv, end - beg)) {
                    hit = true;
                    if (a.hint) a.hint[v] = w[k] | (W ? a.hflag : 0);
                }
                stop |= a.sorted && a.rule == 0 && w[k] >= v;
            }
            const int anyhit = __syncthreads_or(hit);
            const int anystop = __syncthreads_or(stop);
            if (anyhit) {
                lost = true;
                break;
            }
            if (anystop) break;
        }
        if (threadIdx.x == 0) {
            if (lost) {
                const int p = atomicAdd(cnt_out, 1);
                outl[p] = v;
            } else {
                settle<W>(a, v, cv, cmax);
            }
        }
        if (a.pushff && !lost) push_row_coop<W>(a, v, cv, beg, end, threadIdx.x, WG);
    }
}

// Split bucket conflict test: each chunk tests its part of the row (skipped when a
// sibling chunk already found a conflict, or when a sorted chunk starts at w >= v)
// and ORs its verdict into the hub's lost flag; the chunk that completes the
// finished-chunk count settles the hub or requeues it with a fresh chunk range.
template <bool W>
__device__ __forceinline__ void detect_split(const RoundArgs& a, const int* list, int nchunks, int j, int nbk,
                                             RoundLds& s, int* outl, int* cnt_out, int& cmax) {
    const int* cstart = a.cstart[a.par_in];
    const int* owner = a.owner[a.par_in];
    int* cstart_out = a.cstart[a.par_out];
    int* owner_out = a.owner[a.par_out];
    const int tid = threadIdx.x;
    for (int t = j; t < nchunks; t += nbk) {
        const int p = owner[t];
        const int v = list[p];
        const int k = t - cstart[p];
        const int rb = a.rowptr[v], re = a.rowptr[v + 1];
        const int nch = split_chunks(re - rb);
        const int beg = rb + k * SPLIT_CH, end = min(beg + SPLIT_CH, re);
        const int cv = tentative(a, v);
        // the remembered neighbour decides for every chunk of the hub at once
        bool hit = hint_hit(a, v, cv);
        const bool skip = hit || ld_agent(&a.hublost[p]) != 0 ||
                          (a.rule == 0 && a.sorted && a.colidx[beg] >= v);
        if (!skip) {
            const int nq = ((end - beg) + 3 + 3) / 4 + 1;
            for (int q0 = 0; q0 < nq; q0 += WG) {
                int w[4];
                load_quad(a.colidx, a.nnz, beg, end, q0 + tid, w);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    if (loses_to(a, w[kk], v, cv, re - rb)) {
                        hit = true;
                        if (a.hint) a.hint[v] = w[kk] | (W ? a.hflag : 0);
                    }
                }
            }
        }
        const int anyhit = __syncthreads_or(hit);
        if (tid == 0) {
            unsigned old = 0;
            if (anyhit) old = or_agent(reinterpret_cast<unsigned*>(&a.hublost[p]), 1u);
            wait_on(old);
            s.sh[1] = add_agent(&a.hubdone[p], 1) == nch - 1;
        }
        __syncthreads();
        if (s.sh[1]) {
            if (tid == 0) {
                const bool lost = ld_agent(&a.hublost[p]) != 0;
                st_agent(&a.hublost[p], 0);
                st_agent(&a.hubdone[p], 0);
                s.sh[2] = -1;
                if (lost) {
                    const int qn = atomicAdd(cnt_out, 1);
                    const int cs = atomicAdd(&a.ctl->ccnt[a.par_out], nch);
                    outl[qn] = v;
                    cstart_out[qn] = cs;
                    s.sh[2] = qn;
                    s.sh[3] = cs;
                } else {
                    settle<W>(a, v, cv, cmax);
                    s.sh[3] = a.settled ? atomicAdd(&a.ctl->nsettled, nch) : 0;
                }
            }
            __syncthreads();
            if (s.sh[2] >= 0) {
                for (int i = tid; i < nch; i += WG) owner_out[s.sh[3] + i] = s.sh[2];
            } else if (a.settled) {
                // one push task per chunk of the settled row
                for (int i = tid; i < nch; i += WG) {
                    a.settled[s.sh[3] + i] = p;
                    a.settled_k[s.sh[3] + i] = i;
                }
            }
        }
        __syncthreads();
    }
}

// Split bucket with live lists.  Each wavefront takes a batch of up to 64 chunks, one
// lane per chunk.  A lane reads its chunk's record (queue entry, hub, chunk index and
// list slot), then in one step the hub's row bounds, colour word and hint, the chunk's
// list state and the hub's merge word, then the hint's colour word together with the
// first quad of the chunk's list (or unexamined row), and last that quad's colour
// words (live_probe's look, fused).  Only the chunks still undecided then get the
// whole wavefront, one after another (skipped once a sibling chunk has found a
// conflict).  Each lane merges its chunk into the hub's merge word with one 64-bit
// atomic add (the chunk count and, when it found a conflict, one in the high half);
// the chunk that completes the count settles the hub or requeues it with fresh chunks.
template <bool W>
__device__ __forceinline__ void detect_split_wave(const RoundArgs& a, const int* list, int nchunks, int j,
                                                  int nbk, int* outl, int* cnt_out, int& cmax) {
    const int4* crec = a.crec[a.par_in];
    int* cstart_out = a.cstart[a.par_out];
    int* owner_out = a.owner[a.par_out];
    int4* crec_out = a.crec[a.par_out];
    const int lane = __lane_id();
    const int nw = nbk * WAVES;                      // wavefronts of the bucket
    const int gw = j * WAVES + (threadIdx.x >> 6);   // this one's index among them
    // chunks per wavefront: an even share, at most 64 per batch (most chunks need no
    // scan, but the ones that do are scanned one after another).  Wavefront gw takes
    // the chunks s * nw + gw, which spreads the chunks of each hub over the wavefronts
    // (a hub that nothing beats scans every chunk whole)
    const int per = (nchunks + nw - 1) / nw;
    const int hf = W ? a.hflag : 0;
    for (int s0 = 0; s0 < per; s0 += 64) {
        const int t = (s0 + lane) * nw + gw;
        const bool on = s0 + lane < per && t < nchunks;
        int p = 0, v = 0, k = 0, ci = 0;
        if (on) {
            const int4 r = crec[t];
            p = r.x;
            v = r.y;
            k = r.z;
            ci = r.w;
        }
        int rb = 0, re = 0, xv = 0, hh = -1, cl = -1, cp = 0;
        unsigned long long hs = 0;
        if (on) {
            rb = a.rowptr[v];
            re = a.rowptr[v + 1];
            xv = a.X[v];
            hh = a.hint ? a.hint[v] : -1;
            cl = a.clen[ci];
            cp = a.cpos[ci];
            hs = ld_agent(&a.hubst[p]);
        }
        const int cv = xv & CMASK;
        const int nch = split_chunks(re - rb);
        const int beg = rb + k * SPLIT_CH;
        const int end = min(beg + SPLIT_CH, re);
        const int h = (hh != -1 && (a.rule != 0 || (hh & IDMASK) < v)) ? (hh & IDMASK) : -1;
        const bool fresh = cl < 0;                       // nothing examined yet
        const int len = fresh ? 0 : cl;
        const int pos = fresh ? beg : cp;
        const bool empty = len == 0 && pos >= end;        // nothing left to examine
        bool done = !on || (hs >> 32) != 0;              // a sibling chunk found a conflict
        int hx = 0;
        int w[4] = {-1, -1, -1, -1};
        if (!done && h >= 0) hx = a.X[h];
        if (!done && !empty) {
            if (len > 0) load_quad(a.live, a.nnz, beg, beg + len, 0, w);
            else load_quad(a.colidx, a.nnz, pos, end, 0, w);
        }
        bool hit = !done && h >= 0 && (hx & CMASK) == cv;
        int g[4] = {0, 0, 0, 0};
        // entries that beat v: every list entry; of the row, by the rule (degree rule:
        // the neighbours' row bounds are read with their colours)
        bool bt[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bt[q] = w[q] >= 0 && (len > 0 || (a.rule == 0 ? w[q] < v : w[q] != v));
        if (!done && !hit) {
#pragma unroll
            for (int q = 0; q < 4; ++q) g[q] = bt[q] ? a.X[w[q]] : 0;
        }
        if (!done && !hit) {
            int found = -1;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (bt[q] && (g[q] & CMASK) == cv && (len > 0 || a.rule == 0 || beats_v(a, w[q], v, re - rb)))
                    found = w[q];
            if (found >= 0) {
                hit = true;
                if (a.hint) a.hint[v] = found | hf;
            }
        }
        done = done || hit || empty;
        unsigned long long todo = __ballot(!done);
        while (todo) {
            const int jj = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int pj = __builtin_amdgcn_readlane(p, jj);
            // a chunk whose hub another chunk has already decided is skipped
            int sk = 0;
            if (lane == 0) sk = (ld_agent(&a.hubst[pj]) >> 32) != 0;
            if (__builtin_amdgcn_readfirstlane(sk)) continue;
            const int vj = __builtin_amdgcn_readlane(v, jj);
            const int cij = __builtin_amdgcn_readlane(ci, jj);
            const bool hj = live_test_wave(a, vj, __builtin_amdgcn_readlane(re, jj) - __builtin_amdgcn_readlane(rb, jj),
                                           __builtin_amdgcn_readlane(cv, jj), __builtin_amdgcn_readlane(beg, jj),
                                           __builtin_amdgcn_readlane(end, jj), __builtin_amdgcn_readlane(cl, jj),
                                           __builtin_amdgcn_readlane(cp, jj), &a.clen[cij], &a.cpos[cij], hf);
            if (lane == jj) hit = hj;
        }
        // merge: one atomic adds the finished chunk and, with a conflict, a hit
        if (on) {
            const unsigned long long old =
                atomicAdd(&a.hubst[p], 1ull + (hit ? (1ull << 32) : 0ull));
            if ((int)(old & 0xffffffffull) + 1 == nch) {
                // the last chunk to finish settles the hub or requeues it with fresh chunks
                const bool lost = hit || (old >> 32) != 0;
                st_agent(&a.hubst[p], 0ull);
                const int base = ci - k;                 // the hub's chunk slots
                if (lost) {
                    const int qn = atomicAdd(cnt_out, 1);
                    const int cs = atomicAdd(&a.ctl->ccnt[a.par_out], nch);
                    outl[qn] = v;
                    cstart_out[qn] = cs;
                    for (int i = 0; i < nch; ++i) {
                        owner_out[cs + i] = qn;
                        crec_out[cs + i] = make_int4(qn, v, i, base + i);
                    }
                } else {
                    settle<W>(a, v, cv, cmax);
                    if (a.settled) {
                        // one push task per chunk of the settled row
                        const int cs = atomicAdd(&a.ctl->nsettled, nch);
                        for (int i = 0; i < nch; ++i) {
                            a.settled[cs + i] = p;
                            a.settled_k[cs + i] = i;
                        }
                    }
                }
            }
        }
    }
}

// One conflict-test phase for the block `bid` of a grid partitioned by boff.
template <bool W>
__device__ __forceinline__ void detect_phase(const RoundArgs& a, RoundLds& s, int bid, const int* boff, int& cmax) {
    int b, j, nbk;
    block_bucket(boff, bid, b, j, nbk);
    if (bid == 0 && threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < NB; ++k) {
            tot += a.ctl->cnt[a.par_in][k];
            a.ctl->dyn[0][k] = 0;
        }
        // with wake flags the conflict test marks the rounds that test a vertex
        if (tot > 0 && W) a.ctl->rounds = wround_of(a);
        if (tot > 0 && !W) {
            const int ridx = a.ctl->rounds;
            if (a.st_wsize && ridx < a.st_cap) a.st_wsize[ridx] = tot;
            a.ctl->rounds = ridx + 1;
        }
    }
    if (bid >= boff[NB]) return;
    const int cnt = a.ctl->cnt[a.par_in][b];
    const int* list = a.wl_in + a.seg[b];
    int* outl = a.wl_out + a.seg[b];
    int* cnt_out = &a.ctl->cnt[a.par_out][b];
    // Ordered compaction for the buckets that flush per workgroup, when every block's
    // range fits one flush: the block takes a ticket, works on the ticket's range and
    // writes its losers after those of the lower tickets.
    unsigned long long* ust = nullptr;
    if (a.lbs && b <= NTILE && (long long)cnt <= (long long)SUB * nbk) {
        if (threadIdx.x == 0) s.lsh[0] = atomicAdd(&a.ctl->tk[b], 1);
        __syncthreads();
        j = s.lsh[0];
        __syncthreads();
        ust = a.lbs + boff[b];
    }
    const int lo = (int)((long long)j * cnt / nbk);
    const int hi = (int)((long long)(j + 1) * cnt / nbk);
    if (ust && lo >= hi) {
        // an empty range still publishes its (zero) count for the blocks after it
        if (threadIdx.x < 64) lookback(ust, j, 0, &a.ctl->err);
        return;
    }
    if (b < NTILE && a.rule == 0 && !ust && !(a.lane_mode_detect >> 4 & 1)) {
        detect_stream<W, false>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j);
    } else if ((b == NTILE || b == NTILE + 1) && a.live && a.rule == 0 && !ust && !(a.lane_mode_detect >> 5 & 1) &&
               hi - lo >= 64 * WAVES) {
        // long rows, at least 64 per wavefront (the early rounds, whose lists are new and
        // whose conflicts come early): lane-streamed; fewer, with longer lists that the
        // cooperative test keeps compact: detect_wave
        detect_stream<W, true>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j);
    } else if (b < NTILE && (a.lane_mode_detect >> b & 1)) {
        detect_lanes<W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j);
    } else {
        switch (b) {
            case 0: detect_tiles<2, W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j); break;
            case 1: detect_tiles<4, W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j); break;
            case 2: detect_tiles<8, W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j); break;
            case 3: detect_tiles<16, W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j); break;
            case 4: detect_wave<W>(a, list, lo, hi, s, outl, cnt_out, cmax, ust, j); break;
            case 5:
                // with live lists a wavefront per vertex does (the lists shrink quickly)
                if (a.live) detect_wave<W>(a, list, lo, hi, s, outl, cnt_out, cmax, nullptr, 0);
                else detect_wg<W>(a, list, cnt, s, outl, cnt_out, cmax);
                break;
            default:
                if (a.live) detect_split_wave<W>(a, list, a.ctl->ccnt[a.par_in], j, nbk, outl, cnt_out, cmax);
                else detect_split<W>(a, list, a.ctl->ccnt[a.par_in], j, nbk, s, outl, cnt_out, cmax);
                break;
        }
    }
}

// JP rounds have no FirstFit phase, whose first block otherwise clears the output
// queue counters and the conflict-test work counters of the round.
__global__ void k_jp_prep(Ctl* ctl, int par_out, unsigned long long* lbs, int nlbs) {
    const int k = threadIdx.x;
    if (k < NB) {
        ctl->cnt[par_out][k] = 0;
        ctl->dyn[1][k] = 0;
        ctl->tk[k] = 0;
    }
    if (k == 0) ctl->ccnt[par_out] = 0;
    if (lbs)
        for (int i = k; i < nlbs; i += blockDim.x) lbs[i] = 0;
}

// Push phase for the split bucket (push mode): every chunk of a hub that settled this
// round pushes the hub's colour over the chunk's part of the row.
template <bool W>
__device__ __forceinline__ void push_split_phase(const RoundArgs& a, int j, int nbk) {
    const int* list = a.wl_in + a.seg[BSPLIT];
    if (a.settled) {
        // only the chunks of the rows that settled this round, listed by the conflict test
        const int ns = a.ctl->nsettled;
        for (int t = j; t < ns; t += nbk) {
            const int v = list[a.settled[t]];
            const int k = a.settled_k[t];
            const int x = a.X[v];
            const int rb = a.rowptr[v], re = a.rowptr[v + 1];
            const int beg = rb + k * SPLIT_CH, end = min(beg + SPLIT_CH, re);
            push_row_coop<W>(a, v, x, beg, end, threadIdx.x, WG);
        }
        return;
    }
    const int nchunks = a.ctl->ccnt[a.par_in];
    const int* cstart = a.cstart[a.par_in];
    const int* owner = a.owner[a.par_in];
    for (int t = j; t < nchunks; t += nbk) {
        const int p = owner[t];
        const int v = list[p];
        const int x = a.X[v];
        if (x <= 0) continue;                  // requeued: nothing to push
        const int k = t - cstart[p];
        const int rb = a.rowptr[v], re = a.rowptr[v + 1];
        const int beg = rb + k * SPLIT_CH, end = min(beg + SPLIT_CH, re);
        push_row_coop<W>(a, v, x, beg, end, threadIdx.x, WG);
    }
}

template <bool W>
__global__ __launch_bounds__(WG) void k_push(RoundArgs a) { push_split_phase<W>(a, blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// Persistent mode (the kernel fusion of Sec. 3.3): every round of a colouring in
// one launch, FirstFit and the conflict test separated by device-wide barriers.
// The barrier is two-level: blocks first meet on a counter of their XCD group
// (blockIdx mod 8), the last of each group meets the others on a top counter, and
// the last overall advances the generation all blocks wait for.  Counters only grow
// within a run, so no reset is needed between barriers.  The agent-scope fences on
// both sides make the colours and worklists written by one XCD visible to the
// others.
// Every wait is bounded: a block that has waited `limit` wall-clock ticks sets
// ERR_BARRIER and stops waiting, and every block leaves the round loop once that bit
// is set, so a grid that is not fully resident (a plain launch sharing the device with
// another persistent kernel) ends with an error instead of hanging.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void grid_sync(Ctl* ctl, int& gen, long long limit) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x;
        const int ngrp = nblk < 8 ? nblk : 8;
        const int grp = blockIdx.x & 7;
        const int gsize = (nblk - grp + 7) / 8;
        const int target = gen + 1;
        __threadfence();
        const int old = atomicAdd(&ctl->bar[grp][0], 1);
        if (old == gsize * target - 1) {
            const int t = atomicAdd(&ctl->bar_top[0], 1);
            if (t == ngrp * target - 1) __hip_atomic_store(&ctl->bar_gen[0], target, __ATOMIC_RELEASE,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        }
        // spin with relaxed loads (an acquire load would invalidate the L2 on every poll),
        // then one acquire fence
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(&ctl->bar_gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > limit) {
                atomicOr(&ctl->err, ERR_BARRIER);
                break;
            }
        }
        __threadfence();
    }
    gen += 1;
    __syncthreads();
}

// One round of the persistent kernel: FirstFit, barrier, conflict test, barrier, and
// in push mode the split-hub push phase with its barrier.  Returns false when every
// queue was empty (the colouring is complete) or a barrier timed out.
__device__ __forceinline__ bool persistent_round(const RoundArgs& a, RoundLds& s, int* boff, int& total,
                                                 int& gen, int& cmax, long long limit, int r) {
    if (threadIdx.x == 0) {
        int cnt[NB];
        for (int b = 0; b < NB; ++b) cnt[b] = ld_agent(&a.ctl->cnt[a.par_in][b]);
        cnt[BSPLIT] = ld_agent(&a.ctl->ccnt[a.par_in]);
        int t = 0;
        for (int b = 0; b < NB; ++b) t += cnt[b];
        total = (ld_agent(&a.ctl->err) & ERR_BARRIER) ? -1 : t;
        device_plan(cnt, gridDim.x, boff, r);
    }
    __syncthreads();
    if (total <= 0) {
        if (total == 0 && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->pdone = 1;
        return false;
    }
    assign_phase(a, s, blockIdx.x, boff);
    grid_sync(a.ctl, gen, limit);
    detect_phase<false>(a, s, blockIdx.x, boff, cmax);
    grid_sync(a.ctl, gen, limit);
    if (a.pushff && boff[BSPLIT + 1] > boff[BSPLIT]) {
        push_split_phase<false>(a, blockIdx.x, gridDim.x);
        grid_sync(a.ctl, gen, limit);
    }
    return true;
}

// a_odd / a_even: the same arguments with the worklist parities of odd / even round
// indices, used from separate branches (selecting one into a private copy would spill
// its indexed arrays to scratch).  They are constant kernel arguments when the host
// knows every field, or blocks in device memory written by the on-device plan when
// the setup results (bucket segments, row order, arc count) never reach the host.
__device__ __forceinline__ void persistent_rounds(const RoundArgs& a_odd, const RoundArgs& a_even,
                                                  int first_round, int max_rounds, long long limit) {
    __shared__ RoundLds s;
    __shared__ int boff[NB + 1];
    __shared__ int total;
    int gen = 0;
    int cmax = 0;
    for (int r = first_round; r < max_rounds; ++r) {
        const bool more = (r & 1) ? persistent_round(a_odd, s, boff, total, gen, cmax, limit, r)
                                  : persistent_round(a_even, s, boff, total, gen, cmax, limit, r);
        if (!more) break;
    }
    cmax = block_max(cmax, s.red);
    if (threadIdx.x == 0 && cmax > 0) atomicMax(&a_odd.ctl->maxcolor, cmax);
}

__global__ __launch_bounds__(WG) void k_persistent(RoundArgs a_odd, RoundArgs a_even, int first_round,
                                                   int max_rounds, long long limit) {
    persistent_rounds(a_odd, a_even, first_round, max_rounds, limit);
}

}  // namespace csrcolor
