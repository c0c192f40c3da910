/*
 * csrcolor -- speculative-greedy vertex coloring of undirected CSR graphs on
 * AMD Instinct MI355X (gfx950).
 *
 * The library colors a graph with the data-driven speculative-greedy method of
 * Chen et al., "Efficient and High-quality Sparse Graph Coloring on GPUs"
 * (Sec. 3.1, Algorithm Data-GC; FirstFit and ConflictResolve of Sec. 3;
 * colour clearing and worklist push by prefix sum of Sec. 3.1; bitset FirstFit
 * of Sec. 3.2; degree-based load balancing of Sec. 3.3):
 *
 *   W = V; snapshot S = 0 (uncoloured)
 *   repeat until W is empty:
 *     every v in W takes the smallest colour c > 0 not in { S[w] : w in adj(v), w != v }
 *     v in W loses if some neighbour w < v in W took the same colour
 *     winners are fixed in S; losers are cleared and form the next W
 *
 * Rounds are Jacobi-style (FirstFit only sees the previous round's snapshot) and
 * the HIGHER id of a same-colour adjacent pair is requeued, so the result is a
 * deterministic function of the graph: it does not depend on thread timing,
 * launch shape, bucket thresholds or mode.
 *
 * Conventions for every entry point:
 *   - Graphs are symmetric CSR with int32 indices: rowptr[n+1] (rowptr[0] == 0,
 *     non-decreasing) and colidx[rowptr[n]] with entries in [0, n).  Rows need
 *     not be sorted (sorted rows are faster); self-loops are ignored and
 *     duplicate entries are harmless.  Symmetry is a precondition, checked only
 *     when opts->validate >= 1.
 *   - Array arguments are DEVICE pointers owned by the caller unless marked
 *     HOST.  Inputs are only read; outputs must not alias inputs.
 *   - Output colours are 0-based: colors_out[v] in [0, ncolors).
 *   - Work is enqueued on `stream`.  The library keeps a per-(device, stream)
 *     workspace that is grown on demand and freed by csrcolor_release_workspace():
 *     with the default options at most about 56 bytes per vertex plus 5.3 bytes
 *     per arc (colour state, two worklists, conflict hints, live-list lengths,
 *     resume positions and lists, small-colour flag slots, byte flags of the
 *     forbidden colours, wake flags and masks) plus the split-row scratch and a
 *     small control block; the multi-graph call adds a copy of the union CSR and
 *     its colours (csrcolor_workspace_bytes gives the exact bound).  Calls on the
 *     same stream are serialised by a lock, calls on different streams do not
 *     share scratch.
 *   - Errors are negative csrcolor_status values; outputs are then unspecified.
 *     Structural validation (rowptr monotone and in range, colidx in range) is
 *     always done on the device before any colouring kernel runs, so a
 *     malformed graph is reported as CSRCOLOR_EBADCSR, never read out of bounds
 *     (this requires colidx to hold rowptr[n] entries as stated above).
 */
#ifndef CSRCOLOR_H
#define CSRCOLOR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSRCOLOR_OK = 0,
    CSRCOLOR_EINVAL = -1,     /* bad argument: n < 0, NULL pointer with n > 0, bad option */
    CSRCOLOR_EBADCSR = -2,    /* rowptr[0] != 0, rowptr decreasing, or colidx out of [0, n) */
    CSRCOLOR_ENOMEM = -3,     /* device or pinned host allocation failed */
    CSRCOLOR_EHIP = -4,       /* a HIP runtime call failed */
    CSRCOLOR_EOVERFLOW = -5,  /* sizes beyond int32 (batched totals) */
    CSRCOLOR_ENOTSYM = -6,    /* validate >= 1 and the CSR is not symmetric */
    CSRCOLOR_ELIMIT = -7,     /* round limit reached (cannot happen for a valid graph: rounds <= n) */
    CSRCOLOR_ETIMEOUT = -8,   /* a device-wide barrier of the persistent rounds waited more than 8 s:
                                 the grid was not resident (another persistent kernel held the device) */
    CSRCOLOR_ETOOBIG = -9     /* csrcolor_color_noalloc: n or nnz above its fixed maxima */
} csrcolor_status;

/* Fixed maxima of csrcolor_color_noalloc and the size of its scratch array. */
#define CSRCOLOR_NOALLOC_MAX_N       1048576     /* vertices */
#define CSRCOLOR_NOALLOC_MAX_NNZ     33554432    /* arcs (directed entries of colidx) */
#define CSRCOLOR_NOALLOC_SCRATCH_MIB 81          /* device memory per GPU, held until the process ends */

/* How the rounds are driven.  Every mode gives the identical colouring. */
typedef enum {
    CSRCOLOR_MODE_AUTO = 0,        /* library choice */
    CSRCOLOR_MODE_LOOP = 1,        /* host loop: two kernels per round, worklist size read back every few rounds */
    CSRCOLOR_MODE_PERSISTENT = 2,  /* device-planned: the setup results never reach the host and one
                                      kernel runs every round after the first with device-wide
                                      barriers (the kernel fusion of Sec. 3.3); wake flags do not apply */
    CSRCOLOR_MODE_GRAPH = 3        /* blocks of rounds captured once in a hipGraph and replayed (with wake
                                      flags too: the round number is kept on the device) */
} csrcolor_mode;

/* Which endpoint of a same-colour adjacent pair of worklist vertices is requeued. */
typedef enum {
    CSRCOLOR_RULE_ID = 0,      /* the higher vertex id (default) */
    CSRCOLOR_RULE_DEGREE = 1   /* the smaller degree, the higher id on equal degree: the heuristic
                                  conflict resolve of Sec. 3.2 (fewer rounds on skewed graphs) */
} csrcolor_rule;

/* Which colouring method runs. */
typedef enum {
    CSRCOLOR_ALGO_SGR = 0,       /* data-driven speculative greedy with worklists (Sec. 3.1, Algorithm
                                    Data-GC; default) */
    CSRCOLOR_ALGO_SGR_TOPO = 1,  /* topology-driven speculative greedy (Sec. 3.1, Algorithm Topo-GC): every
                                    round visits all n vertices, one lane per vertex.  Same colouring as
                                    CSRCOLOR_ALGO_SGR; kept to measure what the worklists save.  LOOP only */
    CSRCOLOR_ALGO_JP = 2         /* Jones-Plassmann independent sets (Sec. 2.2, Algorithm 3): in round c a
                                    vertex takes colour c iff its priority beats every neighbour still
                                    uncoloured.  The priority of v in round c is output number
                                    c * 2^32 + v of SplitMix64 seeded with seed_hi:seed_lo, compared
                                    unsigned (the map is a bijection, so priorities never tie).  `rule` and `firstfit` are ignored.
                                    LOOP only; not for the batched and multi entry points, because the
                                    priorities depend on vertex ids */
} csrcolor_algorithm;

/* Tuning and checking options.  Zero-initialise and set what you need; every
 * zero field means "library default".  Only `rule`, `algorithm` and (for JP) the
 * seed change the colouring.  A field out of its range, or an algorithm other than
 * CSRCOLOR_ALGO_SGR with mode PERSISTENT or GRAPH (or JP given to the batched or
 * multi entry points), fails the call with CSRCOLOR_EINVAL. */
typedef struct {
    int32_t mode;           /* csrcolor_mode */
    int32_t validate;       /* 1: also check symmetry (sorted rows only; costs one search per arc) */
    int32_t t_wave;         /* max degree handled by one wavefront per vertex (61..1024; default 1024) */
    int32_t t_split;        /* rows longer than this are split over several workgroups (>= 1024; default 2048) */
    int32_t blocks_per_cu;  /* workgroups per compute unit for the round kernels (default 6) */
    int32_t sync_every;     /* LOOP/GRAPH: rounds enqueued between worklist-size read-backs (default 8) */
    int32_t lane_assign;    /* bit b (b < 4): low-degree bucket b runs FirstFit one lane per vertex;
                               0 = default; -1 = none (all use 2/4/8/16 lanes per vertex) */
    int32_t lane_detect;    /* conflict test of the buckets of rows <= 61 arcs: 0 = default: lane-streamed
                               (id rule, unordered compaction: every lane tests its own vertex and takes the
                               next worklist entry as soon as it is decided; otherwise L lanes per vertex);
                               -1 = L lanes per vertex; bit b (b < 4): bucket b one lane per vertex, the
                               wavefront moving on when all 64 are decided (other buckets L lanes) */
    int32_t firstfit;       /* 0: default (push, byte flags); 1: rescan: every FirstFit gathers all neighbour
                               colours (as printed in the paper); 2: push: a vertex that settles marks its
                               colour in per-neighbour flags (bits, set by atomic OR) and FirstFit reads its
                               own flags; 3: push with byte flags (plain stores).  Same colouring */
    int32_t rule;           /* conflict rule, csrcolor_rule; CHANGES the colouring (each rule is exact) */
    int32_t algorithm;      /* csrcolor_algorithm (default CSRCOLOR_ALGO_SGR) */
    uint32_t seed_lo;       /* JP: low and high 32 bits of the 64-bit priority seed */
    uint32_t seed_hi;
    int32_t hints;          /* 0: default (on); 1: on; -1: off.  Conflict hints (id rule): the conflict test
                               first checks the neighbour that requeued the vertex last time and reads the
                               vertex's row only when that one no longer conflicts (same colouring) */
    int32_t live_lists;     /* 0: default (on); 1: on; -1: off.  Live lists (id rule): a vertex of degree > 61
                               tests a list of its lower neighbours that were still uncoloured when last seen,
                               shrunk as they settle, instead of its row (same colouring) */
    int32_t ordered;        /* 0: default (off); 1: on; -1: off.  Order-preserving worklist compaction: blocks
                               take tickets and place their losers after those of lower tickets (look-back
                               prefix), so every worklist keeps ascending id order (same colouring) */
    int32_t wake;           /* 0: default (auto: on when rows longer than 61 arcs hold under a tenth of the
                               arcs); 1: on; -1: off.  Wake flags (id rule, push FirstFit, hints on, LOOP or
                               GRAPH mode, unordered compaction): a requeued vertex is tested again only once its tentative
                               colour or that of the neighbour that requeued it has changed; every other one
                               loses again without being read (same colouring and rounds) */
    int32_t tile_limits;    /* 0: default.  Largest degrees of the tile buckets 0, 1, 2 (2, 4, 8 lanes per vertex
                               in the tiled kernels; bucket 3, 16 lanes, ends at 61 arcs) packed one per byte,
                               t0 | t1 << 8 | t2 << 16 with t0 <= t1 <= t2 and t0 <= 5, t1 <= 13, t2 <= 29 (the
                               defaults 5, 13, 29 are the most each width holds in one quad per lane); smaller
                               values move vertices to wider tiles (same colouring) */
} csrcolor_opts;

/* Optional run statistics (HOST struct).  Set `cap`, `time_kernels` and the array
 * pointers (HOST arrays of `cap` entries, or NULL) before the call; the library
 * fills the rest. */
typedef struct {
    int32_t rounds;         /* out: number of rounds (0 for n == 0) */
    int32_t ncolors;        /* out */
    int32_t rows_sorted;    /* out: 1 if every row was in ascending order */
    int32_t max_degree;     /* out */
    int64_t nnz;            /* out: rowptr[n] */
    int32_t cap;            /* in: capacity of the per-round arrays */
    int32_t time_kernels;   /* in: 1 = time every kernel launch on `stream`: per-round kernels by events
                               that the dispatch itself stamps (hipExtLaunchKernelGGL), setup groups by
                               events recorded around them */
    int64_t *wsize;         /* out: |W_r| for r = 0 .. min(rounds, cap)-1 */
    int64_t *arcs;          /* out: sum of row lengths over W_r (arcs scanned by FirstFit); for
                               CSRCOLOR_ALGO_SGR_TOPO and CSRCOLOR_ALGO_JP only arcs[0] (= rowptr[n]) is
                               filled, later entries are 0 */
    double ms_setup;        /* out (time_kernels): validation and round-1 kernels */
    double ms_assign;       /* out (time_kernels): all FirstFit kernel launches */
    double ms_detect;       /* out (time_kernels): all conflict-test kernel launches */
    int32_t n_assign;       /* out (time_kernels): FirstFit launches */
    int32_t n_detect;       /* out (time_kernels): conflict-test launches */
    int64_t *kernel_bytes;  /* in: NULL, or a HOST array of 2 filled on return: the bytes moved (each element
                               read or written counted once, at its size) by all recolouring FirstFit launches
                               and all flag-scanning conflict-test launches of a run with wake flags (0 for
                               other runs).  Counting runs slower kernels: request it apart from timing */
} csrcolor_stats;

/* Colour one graph (Sec. 3.1, Algorithm Data-GC).
 *   n          number of vertices (>= 0)
 *   rowptr     DEVICE int32[n+1]
 *   colidx     DEVICE int32[rowptr[n]] (may be NULL when rowptr[n] == 0)
 *   colors_out DEVICE int32[n], written with 0-based colours
 *   ncolors    HOST int32*, receives the number of colours (max colour + 1; 0 if n == 0)
 *   stream     HIP stream; the call synchronises it before returning.
 * Returns CSRCOLOR_OK or a negative csrcolor_status. */
int csrcolor_color(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                   int32_t *colors_out, int32_t *ncolors, hipStream_t stream);

/* Colour one graph with options and statistics (Sec. 3.1, Algorithm Data-GC), as the
 * boundary of an asynchronous caller: the colour count goes to device memory.
 *   n            number of vertices (>= 0)
 *   rowptr       DEVICE int32[n+1];  colidx DEVICE int32[rowptr[n]];  colors_out DEVICE int32[n]
 *   ncolors_dev  DEVICE int32* (may be NULL): receives the number of colours, or, when the device
 *                finds the input or the run at fault, the negative csrcolor_status (EBADCSR,
 *                ENOTSYM, EINVAL, ENOMEM, ETIMEOUT, ELIMIT)
 *   opts         NULL for defaults
 *   stats        NULL, or a HOST struct filled on return
 * Asynchronous (device-planned) when opts->mode is CSRCOLOR_MODE_PERSISTENT, or AUTO with
 * stats == NULL and the SGR algorithm: the call enqueues every kernel on `stream` and returns
 * without waiting and without host<->device copies, so it can be captured into a hipGraph and
 * replayed.  Only the first call on a stream, and a call whose n exceeds every earlier one on
 * that stream, reads rowptr[n] back to size the workspace (that call waits; make it before a
 * capture).  A later graph with more arcs than the workspace was sized for fails on the device
 * with CSRCOLOR_ENOMEM in *ncolors_dev (any synchronous call on the stream, or an asynchronous
 * call with more vertices, sizes it again).  The run uses one persistent kernel whose
 * workgroups must all be resident: outside a capture it is a cooperative launch; inside a
 * capture it is a plain launch, which assumes that no other persistent kernel shares the
 * device while the graph runs (else the run ends with CSRCOLOR_ETIMEOUT, it does not hang).
 * With stats != NULL, or another mode, the call waits for the stream before returning (host-
 * driven modes: LOOP, GRAPH, and AUTO with statistics), and *ncolors_dev is written before it
 * returns.  Host-detected errors (bad arguments, allocation or launch failures) are returned.
 * Speed: the persistent kernel's device-wide barriers cost more than kernel boundaries, so on
 * large skewed graphs the asynchronous path is slower than the host loop (measured on MI355X,
 * R-MAT scale 23: 81 ms against 40 ms for csrcolor_color); on small graphs it is the faster
 * one (no host round trips; ER 16K: 0.32 ms, 0.30 ms replayed from a captured graph). */
int csrcolor_color_ex(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                      int32_t *colors_out, int32_t *ncolors_dev,
                      const csrcolor_opts *opts, csrcolor_stats *stats, hipStream_t stream);

/* For callers that cannot allocate device or host memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): csrcolor_color_ex's asynchronous
 * (device-planned) colouring with default options, over a fixed scratch array that the
 * library holds in device memory (CSRCOLOR_NOALLOC_SCRATCH_MIB MiB per GPU it runs on,
 * from the library's load until the process ends) instead of a workspace it allocates.
 * The call makes no allocation (no hipMalloc, hipHostMalloc, hipFree or allocating
 * library routine), no host<->device copy and no wait: it enqueues the validation, the
 * round-1 kernel, one persistent round kernel (a plain launch of no more workgroups than
 * fit on the device at once) and the kernel that writes the count, so it can be captured
 * into a hipGraph.  Live lists are off; the colouring is csrcolor_color_ex's (the same
 * for every option).
 *   n            number of vertices, 0 <= n <= CSRCOLOR_NOALLOC_MAX_N
 *   nnz          number of arcs, 0 <= nnz <= CSRCOLOR_NOALLOC_MAX_NNZ; must equal rowptr[n]
 *                (checked on the device before any colidx entry is read: EBADCSR)
 *   rowptr       DEVICE int32[n+1];  colidx DEVICE int32[nnz];  colors_out DEVICE int32[n]
 *   ncolors_dev  DEVICE int32* (may be NULL): the number of colours, or the negative status
 *                the device found (EBADCSR, ETIMEOUT)
 * Returns CSRCOLOR_ETOOBIG (nothing enqueued) when n or nnz exceed the maxima, EINVAL for
 * bad arguments, EHIP when a launch fails.  Every call on one GPU shares that GPU's
 * scratch array and leaves its contents there (each call clears what must start at
 * zero): calls whose work overlaps on one GPU (different streams, or host threads
 * without ordering) race and give undefined results; order them on one stream. */
int csrcolor_color_noalloc(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                           int32_t *colors_out, int32_t *ncolors_dev, hipStream_t stream);

/* Colour G independent graphs stored as one block-diagonal CSR with global ids
 * (graph g owns vertices voff[g] .. voff[g+1]-1; its arcs must stay inside that
 * range).  Because rounds only look at neighbours and the requeue rule is
 * invariant under a constant id shift, every graph receives exactly the colouring
 * it would receive alone.
 *   G            number of graphs (>= 0)
 *   n_total      total vertices (must equal voff[G])
 *   voff         DEVICE int64[G+1], voff[0] == 0, non-decreasing
 *   rowptr       DEVICE int32[n_total+1]
 *   colidx       DEVICE int32[rowptr[n_total]], global ids
 *   colors_out   DEVICE int32[n_total], 0-based colours local to each graph
 *   ncolors_out  DEVICE int32[G], colours used by each graph
 *   opts         NULL for defaults
 * With opts->mode == CSRCOLOR_MODE_PERSISTENT the whole union is coloured device-planned in
 * one persistent launch (the kernel fusion of Sec. 3.3) and the call returns without waiting,
 * as csrcolor_color_ex does: a device-detected error then puts the negative status in every
 * ncolors_out entry.  Every other mode synchronises `stream` before returning. */
int csrcolor_color_batched(int32_t G, int32_t n_total, const int64_t *voff,
                           const int32_t *rowptr, const int32_t *colidx,
                           int32_t *colors_out, int32_t *ncolors_out,
                           const csrcolor_opts *opts, hipStream_t stream);

/* Colour G separate graphs in one run (request batching).  The library copies the
 * graphs, ids shifted, into one block-diagonal CSR it owns, colours that union as in
 * csrcolor_color_batched (every graph gets exactly its stand-alone colouring) and
 * copies each graph's colours to its own output.
 *   G            number of graphs (>= 0)
 *   n_host       HOST int32[G]: vertices of graph g
 *   nnz_host     HOST int64[G]: arcs of graph g (must equal rowptr_g[n_g])
 *   rowptr_host  HOST array of G DEVICE pointers, graph g's int32[n_g+1] (rowptr_g[0] == 0)
 *   colidx_host  HOST array of G DEVICE pointers, graph g's int32[nnz_g] with local ids
 *   colors_host  HOST array of G DEVICE pointers, graph g's int32[n_g] output
 *   ncolors_out  DEVICE int32[G]
 *   opts         NULL for defaults
 * Totals must fit int32 (else CSRCOLOR_EOVERFLOW).  A graph whose rowptr does not start
 * at 0 or end at nnz_g, or whose ids leave [0, n_g), fails the call with
 * CSRCOLOR_EBADCSR.  The call synchronises `stream` before returning. */
int csrcolor_color_multi(int32_t G, const int32_t *n_host, const int64_t *nnz_host,
                         const int32_t *const *rowptr_host, const int32_t *const *colidx_host,
                         int32_t *const *colors_host, int32_t *ncolors_out,
                         const csrcolor_opts *opts, hipStream_t stream);

/* Upper bound, in bytes, of the device memory one workspace needs to colour a graph of
 * n vertices and nnz arcs with any options except statistics and ordered compaction
 * (csrcolor_color, _ex, _batched; for csrcolor_color_multi give G >= 1 and the union's
 * totals: it adds the library's copy of the union).  A workspace is kept per (device,
 * stream) at the largest size it has needed, so a caller that bounds the graphs it
 * gives one stream bounds that stream's workspace.  Pinned host staging (a few bytes
 * per graph) is not included.  Returns CSRCOLOR_EINVAL for negative arguments. */
int64_t csrcolor_workspace_bytes(int32_t G, int64_t n, int64_t nnz);

/* Device bytes the library's workspaces hold now, over every device and stream (the
 * fixed array of csrcolor_color_noalloc excluded).  Must not overlap a call that grows
 * or releases a workspace. */
int64_t csrcolor_device_bytes_in_use(void);

/* Static description of a status code. */
const char *csrcolor_strerror(int status);

/* Free every library-owned workspace on every device.  Must not overlap a
 * running call. */
void csrcolor_release_workspace(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int csrcolor_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSRCOLOR_H */
