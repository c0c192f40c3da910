// Device-side building blocks for speculative-greedy colouring on gfx950.
//
// Colour state: one int32 per vertex, X[v]:
//   X[v] > 0                 v is settled with colour X[v] (1-based)
//   X[v] == 0 or X[v] < 0    v is uncoloured in the snapshot; a negative value is
//                            FLAG | c, the tentative colour c of the current round
//                            (with wake flags also BIG when v has more than WAKE_DEG arcs).
// FirstFit reads only X[w] > 0 (the previous round's snapshot) and writes FLAG|c
// for its own worklist vertex; the conflict test compares colour parts
// (X & CMASK), so the value a neighbour holds before or after its own write in the
// same phase gives the same answer.  This folds the snapshot array and the
// tentative array of the round definition (Sec. 3.1, Algorithm Data-GC with
// colour clearing) into one array without any ordering hazard inside a phase.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csrcolor {

constexpr int WG = 256;               // threads per workgroup (4 wavefronts of 64)
constexpr int WAVES = WG / 64;
constexpr int NB = 7;                 // degree buckets
constexpr int FLAG = (int)0x80000000;
constexpr int BIG = 0x40000000;       // wake flags: marks the tentative colour of a row longer than WAKE_DEG
constexpr int CMASK = 0x3fffffff;     // colour part of a colour word (colours stay below 2^30)
constexpr int IDMASK = 0x7fffffff;    // vertex id part of a conflict hint
constexpr int WAVE_CAP = 512;         // per-wavefront loser buffer (LDS entries)
constexpr int SUB = WAVES * WAVE_CAP; // worklist entries per LDS flush
constexpr int OVW = 32;               // overflow bitmap words per wavefront (colours 65..1088)
constexpr int TWAVE_MIN = 61;         // t_wave = 61 leaves the wavefront bucket empty
constexpr int TWAVE_MAX = 1024;       // largest degree handled by one wavefront
constexpr int TSPLIT_MIN = 1024;      // rows above t_split are split (t_split >= t_wave)
constexpr int BMW = 1024;             // workgroup bitmap words (32768 colours per window)
constexpr int AU = 2;                 // arc-loop unroll of the wavefront / workgroup buckets

// Degree buckets.  Buckets 0..3 are "tile" buckets: L = 2, 4, 8, 16 lanes per vertex,
// each lane reading one aligned 16-byte quad of the row, so a row of degree
// <= 4L - 3 is covered whatever its alignment: degrees 1-5, 6-13, 14-29, 30-61.
// Bucket 4: one wavefront per vertex (62 .. t_wave); bucket 5: one workgroup per
// vertex (t_wave .. t_split); bucket 6: rows split into SPLIT_CH-arc chunks, one
// workgroup per chunk.  Degree-0 vertices settle in round 1 and are never queued.
constexpr int NTILE = 4;
constexpr int BSPLIT = 6;
constexpr int SPLIT_CH = 2048;        // arcs per chunk of a split row
constexpr int HW = 32;                // words of a split row's colour bitmap (colours 1..1024)
// Largest degrees of the tile buckets 0..2 packed one per byte (bucket 3 ends at 61):
// the defaults are the most each tile width can hold (4L-3 for L = 2, 4, 8 lanes); any
// smaller non-decreasing values are valid and only move vertices to wider tiles.
constexpr int TILES_DEFAULT = 5 | (13 << 8) | (29 << 16);
__host__ __device__ inline int bucket_of(int deg, int tiles, int twave, int tsplit) {
    return deg <= (tiles & 0xff) ? 0 : deg <= ((tiles >> 8) & 0xff) ? 1 : deg <= ((tiles >> 16) & 0xff) ? 2
         : deg <= 61 ? 3 : deg <= twave ? 4 : deg <= tsplit ? 5 : 6;
}
__host__ __device__ inline int split_chunks(int deg) { return (deg + SPLIT_CH - 1) / SPLIT_CH; }

// Does neighbour w (same tentative colour) requeue v?  dv = deg(v).
__device__ __forceinline__ bool beats(int rule, const int* __restrict__ rowptr, int w, int v, int dv) {
    if (rule == 0) return w < v;
    const int dw = rowptr[w + 1] - rowptr[w];
    return dw > dv || (dw == dv && w < v);
}

// Conflict of v (tentative colour cv, degree dv) with row entry w (-1 = none).
// Under the id rule only lower ids are gathered.
__device__ __forceinline__ bool conflict(int rule, const int* __restrict__ rowptr, const int* X, int w, int v,
                                         int cv, int dv) {
    if (w < 0 || w == v) return false;
    if (rule == 0) return w < v && (X[w] & CMASK) == cv;
    return (X[w] & CMASK) == cv && beats(1, rowptr, w, v, dv);
}

// Wake flags: a vertex sleeps only when it and the neighbour that beat it have at most
// WAKE_DEG arcs (the tile buckets), so waking the sleepers of a recoloured vertex reads
// a short row; every other requeued vertex is awake (tested every round).
constexpr int WAKE_DEG = 61;

// Push FirstFit with byte flags keeps the forbidden colours 1..KQ of every vertex in a
// slot of KQ bytes of its own (Fq[v*KQ + c-1]): a push of such a colour is a single
// store, with no read of the neighbour's row bounds, and FirstFit reads the slot in one
// 16-byte load.  Higher colours use the flags at rowptr[v]+v+c-1 of F.
constexpr int KQ = 16;

// Where a settling vertex pushes its colour (push-mode FirstFit).
struct PushCtx {
    unsigned* F;                  // forbidden-colour flags (bits, or bytes when `bytes`)
    unsigned char* Fq;            // byte flags: the slots of colours 1..KQ (nullptr: off)
    const int* rowptr;
    const int* colidx;
    int nnz;
    bool bytes;
    unsigned char* dirty;         // nullptr, or per-vertex "flags changed" bytes
    // wake flags (rflag == nullptr: off): a neighbour whose tentative colour is the
    // pushed colour must take a new one next round, so its recolour flag is set
    const int* X;
    unsigned char* rflag;
    // wake flags: the forbidden colours 1..64 of a vertex of at most WAKE_DEG arcs as one
    // 64-bit mask (bit c-1), set by atomic OR; longer rows keep their flags in F
    unsigned long long* Fs;
    bool all_tentative;           // round 1: every neighbour of a winner holds colour 1
    long long* nbytes;            // nullptr, or the calling thread's count of bytes moved
    bool loaded;                  // the colidx entries were already read (not counted again)
};

// Marks colour c among the forbidden colours of neighbour u (push-mode FirstFit).
// Only colours <= deg(u)+1 can change u's smallest free colour, and only they have a
// flag: flag c-1 of u sits at position rowptr[u]+u+c-1, one bit of F (set with an
// atomic OR, several neighbours may share a word) or, with `bytes`, one byte (a plain
// store: concurrent writers of one byte all write 1, and distinct bytes of a line are
// merged by the caches).
// With `dirty`, u is also marked for its next FirstFit (a vertex whose flags did not
// change keeps its tentative colour, and FirstFit skips it).
// With wake flags a settled neighbour is skipped (its flags are never read again), and
// a neighbour holding tentative colour c gets its recolour flag (its smallest free
// colour moves); concurrent writers all store 1.
__device__ __forceinline__ void push_flag(const PushCtx& P, int u, int c, int ub, int ue) {
    if (c - 1 <= ue - ub) {
        const long long pos = (long long)ub + u + c - 1;
        if (P.bytes) {
            reinterpret_cast<unsigned char*>(P.F)[pos] = 1;
        } else {
            atomicOr(&P.F[pos >> 5], 1u << (pos & 31));
        }
        if (P.dirty) P.dirty[u] = 1;
    }
}
// A push reads one thing of the neighbour u first (with wake flags its colour word,
// else its rowptr pair) and then writes its flags.  The two halves are separate so that
// a lane pushing to several neighbours issues all the reads before any write: a read
// that follows a write waits for the write too (the vector memory counter covers both),
// and the writes are atomics or stores that go to memory.  (With small-colour slots
// push_quad does its own reads.)
struct PushRead {
    int a;   // wake flags (not round 1): u's colour word; else rowptr[u]
    int b;   // rowptr[u + 1] (not read with wake flags)
};
__device__ __forceinline__ PushRead push_read(const PushCtx& P, int u) {
    PushRead r;
    if (P.rflag && !P.all_tentative) {
        r.a = P.X[u];
        r.b = 0;
    } else {
        r.a = P.rowptr[u];
        r.b = P.rowptr[u + 1];
    }
    return r;
}
__device__ __forceinline__ void push_write(const PushCtx& P, int u, int c, PushRead r) {
    if (P.rflag && !P.all_tentative) {
        // wake flags: the colour word says whether u is settled, short (mask) or long
        const int xu = r.a;
        if (P.nbytes) *P.nbytes += (P.loaded ? 0 : 4) + 4;   // colidx entry, colour
        if (xu > 0) return;
        if (xu & BIG) {
            const int ub = P.rowptr[u];
            const int ue = P.rowptr[u + 1];
            push_flag(P, u, c, ub, ue);
            if (P.nbytes) *P.nbytes += 8 + (c - 1 <= ue - ub ? 1 : 0);
        } else if (c <= 64) {
            // colours above 64 cannot be the smallest free colour of u (at most 62)
            atomicOr(&P.Fs[u], 1ull << (c - 1));
            if (P.nbytes) *P.nbytes += 8;
        }
        if ((xu & (FLAG | CMASK)) == (FLAG | c)) {
            P.rflag[u] = 1;
            if (P.nbytes) *P.nbytes += 1;
        }
        return;
    }
    const int ub = r.a;
    const int ue = r.b;
    if (P.nbytes) *P.nbytes += (P.loaded ? 8 : 12);   // colidx entry, rowptr pair
    if (P.rflag) {
        // round 1 with wake flags: every neighbour of a winner is a loser holding colour 1;
        // a short one keeps its forbidden colours in its mask (all writers store 1)
        P.rflag[u] = 1;
        if (ue - ub <= WAKE_DEG) P.Fs[u] = 1ull;
        else push_flag(P, u, c, ub, ue);
        return;
    }
    push_flag(P, u, c, ub, ue);
}

// Holds the wavefront here until x is loaded.  Placed after a group of reads and before
// the writes that use them, it makes the one wait cover every read of the group: the
// compiler otherwise waits again before each later use inside the writes' branches, and
// such a wait also waits for every write issued before it.
__device__ __forceinline__ void reads_done(int x) { asm volatile("" ::"v"(x)); }

// Pushes colour c of v to the neighbours w[0..3] (entries -1 and v itself are skipped),
// all four reads first.  With small-colour slots a colour <= KQ is one store per
// neighbour; a higher one reads the neighbours' colour words first and only the
// uncoloured ones' row bounds (a settled neighbour never runs FirstFit again, so its
// flags are not needed).
__device__ __forceinline__ void push_quad(const PushCtx& P, const int* w, int v, int c) {
    if (P.Fq && !P.rflag) {
        bool go[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) go[k] = w[k] >= 0 && w[k] != v;
        if (c <= KQ) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (go[k]) P.Fq[(size_t)w[k] * KQ + c - 1] = 1;
            return;
        }
        int x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = go[k] ? P.X[w[k]] : 1;
        reads_done(x[0] | x[1] | x[2] | x[3]);
        int ub[4], ue[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            go[k] = go[k] && x[k] <= 0;
            ub[k] = go[k] ? P.rowptr[w[k]] : 0;
            ue[k] = go[k] ? P.rowptr[w[k] + 1] : 0;
        }
        reads_done(ub[0] | ub[1] | ub[2] | ub[3] | ue[0] | ue[1] | ue[2] | ue[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (go[k]) push_flag(P, w[k], c, ub[k], ue[k]);
        return;
    }
    PushRead r[4];
    int all = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[k].a = 1;
        r[k].b = 0;
        if (w[k] >= 0 && w[k] != v) r[k] = push_read(P, w[k]);
        all |= r[k].a | r[k].b;
    }
    reads_done(all);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (w[k] >= 0 && w[k] != v) push_write(P, w[k], c, r[k]);
}

// Internal rule number of the Jones-Plassmann independent-set colouring (Sec. 2.2,
// Algorithm 3): in round c a worklist vertex takes colour c iff its priority exceeds
// that of every neighbour still uncoloured (colour 0) or coloured this round (c).
constexpr int RULE_JP = 2;

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number k of the generator
// seeded with s is the published output function applied to s + k * golden gamma.
__host__ __device__ __forceinline__ unsigned long long splitmix64(unsigned long long s, unsigned long long k) {
    unsigned long long z = s + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// JP priority of vertex v in round c: output number c * 2^32 + v, compared unsigned.
__host__ __device__ __forceinline__ unsigned long long jp_prio(unsigned long long seed, int c, int v) {
    return splitmix64(seed, ((unsigned long long)(unsigned)c << 32) + (unsigned)v);
}

// Bits of Ctl::err.  The host maps them to a status: ROWPTR, COLIDX, MULTI and
// BATCH to CSRCOLOR_EBADCSR, ASYM to CSRCOLOR_ENOTSYM, UNSORTED to CSRCOLOR_EINVAL,
// NOMEM to CSRCOLOR_ENOMEM, BARRIER to CSRCOLOR_ETIMEOUT, the others to CSRCOLOR_EHIP.
constexpr int ERR_ROWPTR = 1;      // rowptr not monotone from 0 within [0, rowptr[n]]
constexpr int ERR_COLIDX = 2;      // a colidx entry outside [0, n)
constexpr int ERR_ASYM = 4;        // symmetry check failed
constexpr int ERR_INTERNAL = 8;
constexpr int ERR_LOOKBACK = 16;   // an ordered-compaction look-back gave up
constexpr int ERR_MULTI = 32;      // multi-graph call: a graph's rowptr does not span [0, nnz_g]
constexpr int ERR_BATCH = 64;      // batched call: bad vertex offsets or an arc leaving its graph
constexpr int ERR_UNSORTED = 128;  // the symmetry check was asked for on unsorted rows
constexpr int ERR_BARRIER = 256;   // a device-wide barrier of the persistent rounds timed out
constexpr int ERR_NOMEM = 512;     // device-planned run: the graph needs more scratch than was given

// Device-resident control block.
struct Ctl {
    int cnt[2][8];      // worklist length per bucket, double-buffered by round parity
    int dyn[2][8];      // dynamic work counters for workgroup-per-vertex buckets (per phase)
    int hist[8];        // vertices per degree bucket (deg >= 1)
    int maxcolor;       // largest settled colour
    int err;            // bit 0: rowptr, bit 1: colidx range, bit 2: asymmetric, bit 3: internal,
                        // bit 4: a look-back walk gave up
    int desc_total;     // positions e >= 1 with colidx[e] < colidx[e-1]
    int desc_bound;     // such positions that start a non-empty row
    int maxdeg;
    int rounds;         // number of non-empty rounds so far (wake flags: the last round
                        // whose conflict test found a vertex to test)
    int nnz;            // rowptr[n]
    int hchunks;        // chunks over all split-bucket vertices
    int ccnt[2];        // chunks queued in the split bucket, by round parity
    int pdone;          // persistent mode: set when a round found every queue empty
    int tk[8];          // ordered compaction: conflict-test tickets per bucket (reset by FirstFit)
    int tk1;            // ordered compaction: round-1 tickets
    int nsettled;       // push tasks (split row, chunk) of the rows that settled this round
    int pround;         // FirstFit phases run so far (the 0-based index of the current round)
    int wr;             // wake-flag rounds replayed from a captured graph (advanced by k_wassign)
    long long bigarcs;  // arcs of the rows longer than WAKE_DEG
    // device-wide barrier of the persistent mode, each counter on its own 128-byte line
    int bar[8][32];
    int bar_top[32];
    int bar_gen[32];
};

struct Seg {
    int s[NB + 1];
};

struct RoundArgs {
    int n;
    const int* __restrict__ rowptr;
    const int* __restrict__ colidx;
    int* X;
    int* out;
    const int* wl_in;
    int* wl_out;
    Ctl* ctl;
    int par_in;         // worklist parity read this round
    int par_out;
    int twave;
    int tiles;          // tile-bucket degree limits (bucket_of)
    int sorted;         // 1: every row ascending -> conflict scans stop at the first w >= v
    int round;          // persistent mode: 0-based index of the first round it runs
    int nnz;            // rowptr[n], bounds the 16-byte row reads
    int lane_mode_assign;  // bit b: tile bucket b runs FirstFit lane-per-vertex
    int lane_mode_detect;  // bit b: tile bucket b runs the conflict test lane-per-vertex
    int tsplit;            // largest degree handled without splitting the row
    int dev_plan;          // 1: every block derives the bucket partition from the device queue sizes
    // push mode: F holds, for every vertex v, deg(v)+1 bits starting at bit rowptr[v]+v;
    // bit c-1 set <=> a neighbour settled with colour c in an earlier round
    int pushff;         // 0: rescan FirstFit; 1: push, bit flags; 2: push, byte flags
    unsigned* F;
    // push mode: dirty[v] = 1 when a flag of v was set since its last FirstFit
    unsigned char* dirty;
    // conflict rule: 0 = the higher id is requeued; 1 = the smaller degree (row
    // length) is requeued, the higher id on equal degree (heuristic of Sec. 3.2)
    int rule;
    // conflict hints (id rule only; nullptr = off): hint[v] is a neighbour that beat v
    // in an earlier round; the test checks it first and reads v's row only if it no
    // longer conflicts
    int* hint;
    // live lists (id rule; nullptr = off): for a vertex of degree > 61 the lower
    // neighbours found still uncoloured when last seen, packed at live[rowptr[v] ...];
    // llen[v] = their number (-1: nothing examined yet) and lpos[v] = the first row
    // entry no test has examined; for a split row llen[v] is instead the base of its
    // per-chunk lengths clen[llen[v] + k] (-1: nothing examined yet) and resume
    // positions cpos[llen[v] + k]
    int* live;
    int* llen;
    int* clen;
    int* lpos;
    int* cpos;
    // push FirstFit with byte flags (not with wake flags): per vertex KQ bytes for the
    // forbidden colours 1..KQ (nullptr = off)
    unsigned char* Fq;
    // ordered compaction (nullptr = off): one look-back status word per block of the
    // grid, cleared by the FirstFit launch of the round
    unsigned long long* lbs;
    int lbs_n;          // status words to clear: the conflict-test grid size
    // JP (rule RULE_JP): this round's colour and the priority generator's seed
    int jpc;
    unsigned long long seed;
    // split bucket: per queued hub its first chunk; per chunk the hub's queue entry;
    // per queue entry a colour bitmap, a finished-chunk counter and a lost flag
    int* cstart[2];
    int* owner[2];
    unsigned* hubbm;
    int* hubdone;
    int* hublost;
    // split bucket with live lists: per chunk its record {queue entry, hub, chunk index,
    // list slot}; per queue entry one word holding the finished-chunk count (low half)
    // and the number of chunks that found a conflict (high half)
    int4* crec[2];
    unsigned long long* hubst;
    int* settled;       // push tasks of the split rows that settled this round: queue entry
    int* settled_k;     // and chunk index
    // wake flags (rflag != nullptr): a requeued vertex of at most WAKE_DEG arcs is
    // tested again only when its tentative colour or that of the neighbour that beat it
    // (its hint) has changed, or every round while awake; longer ones stay on the
    // worklists.  rflag[v]: recolour v this round (set by pushes); aflag[v]: test v
    // this round (set by recolouring, kept by an awake loser); srnd[v]: the round v
    // settled in; wround: this round's number, or with wround_dev != nullptr one more than
    // the count there (rounds replayed from a captured graph: the recolouring FirstFit
    // advances it)
    int wround;
    const int* wround_dev;
    unsigned char* rflag;
    unsigned char* aflag;
    int* srnd;
    int hflag;          // FLAG with wake flags (a long row's hint never names it a sleeper), else 0
    unsigned long long* Fs;   // wake flags: forbidden-colour masks of the rows of at most WAKE_DEG arcs
    int gdense;         // blocks of the flag-scanning grids
    int vpw;            // vertices per wavefront in the flag scans (64, 128, 256 or 512)
    // nullptr, or bytes moved (algorithmic, each element at its size) by the recolouring
    // and the flag-scanning test launches: [0] and [1], summed over the run
    unsigned long long* ubytes;
    int st_cap;
    long long* st_wsize;
    long long* st_arcs;
    int seg[NB + 1];    // bucket segment offsets inside the worklist arrays
    int boff[NB + 1];   // block offsets of each bucket inside the grid
};

// The number of the current wake-flag round, for the kernels after the recolouring
// FirstFit of the round (which advances the device count when rounds are replayed from
// a captured graph).
__device__ __forceinline__ int wround_of(const RoundArgs& a) {
    return a.wround_dev ? *a.wround_dev + 1 : a.wround;
}

// Tentative colour of worklist vertex v: the FirstFit result in X, or under JP the
// colour of the round.
__device__ __forceinline__ int tentative(const RoundArgs& a, int v) {
    return a.rule == RULE_JP ? a.jpc : (a.X[v] & CMASK);
}

// Does the remembered neighbour of worklist vertex v still requeue it?  A neighbour
// that settled in an earlier round cannot hold v's tentative colour (FirstFit excluded
// it), so an equal colour part means a worklist neighbour of this round that beats v:
// the same verdict the full scan would reach.  (The hint was recorded because it beat
// v, and neither ids nor degrees change, so under either rule it still beats v.)
// With wake flags the hint of a vertex of at most WAKE_DEG arcs carries FLAG when the
// neighbour has more arcs (no hint is -1).
__device__ __forceinline__ bool hint_hit(const RoundArgs& a, int v, int cv) {
    if (!a.hint) return false;
    const int h = a.hint[v];
    return h != -1 && (a.rule != 0 || (h & IDMASK) < v) && (a.X[h & IDMASK] & CMASK) == cv;
}

// Is worklist vertex v (tentative colour cv, degree dv) requeued because of row entry
// w (-1 = none)?  SGR rules: same tentative colour and w beats v.  JP: w is still
// competing this round and v's priority does not exceed w's (a tie blocks both).
__device__ __forceinline__ bool loses_to(const RoundArgs& a, int w, int v, int cv, int dv) {
    if (a.rule != RULE_JP) return conflict(a.rule, a.rowptr, a.X, w, v, cv, dv);
    if (w < 0 || w == v) return false;
    const int xw = a.X[w];
    return (xw == 0 || xw >= cv) && jp_prio(a.seed, cv, v) <= jp_prio(a.seed, cv, w);
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const int l = __lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

template <int G>
__device__ __forceinline__ unsigned long long group_or(unsigned long long m) {
    unsigned lo = (unsigned)m, hi = (unsigned)(m >> 32);
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
        lo |= __shfl_xor(lo, off, 64);
        hi |= __shfl_xor(hi, off, 64);
    }
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
    return x;
}

// Exclusive prefix over the wavefront's lanes of c; `total` receives the sum.
__device__ __forceinline__ int wave_excl(int c, int& total) {
    const int lane = __lane_id();
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    total = __shfl(incl, 63, 64);
    return incl - c;
}

__device__ __forceinline__ long long wave_sum64(long long x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned lo = (unsigned)x, hi = (unsigned)((unsigned long long)x >> 32);
        lo = __shfl_xor(lo, off, 64);
        hi = __shfl_xor(hi, off, 64);
        x += (long long)(((unsigned long long)hi << 32) | lo);
    }
    return x;
}

// Block-wide reductions through a small LDS scratch (every thread must call).
__device__ __forceinline__ int block_max(int x, int* s) {
    x = wave_max(x);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) s[wv] = x;
    __syncthreads();
    int r = s[0];
#pragma unroll
    for (int k = 1; k < WAVES; ++k) r = max(r, s[k]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_min(int x, int* s) {
    x = wave_min(x);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) s[wv] = x;
    __syncthreads();
    int r = s[0];
#pragma unroll
    for (int k = 1; k < WAVES; ++k) r = min(r, s[k]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_sum(int x, int* s) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) s[wv] = x;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) r += s[k];
    __syncthreads();
    return r;
}

__device__ __forceinline__ long long block_sum64(long long x, long long* s) {
    x = wave_sum64(x);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) s[wv] = x;
    __syncthreads();
    long long r = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) r += s[k];
    __syncthreads();
    return r;
}

}  // namespace csrcolor
