// Device-side building blocks for speculative-greedy colouring on gfx950.
//
// Colour state: one int32 per vertex, X[v]:
//   X[v] > 0                 v is settled with colour X[v] (1-based)
//   X[v] == 0 or X[v] < 0    v is uncoloured in the snapshot; a negative value is
//                            FLAG | c, the tentative colour c of the current round.
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
constexpr int NB = 5;                 // degree buckets
constexpr int FLAG = (int)0x80000000;
constexpr int CMASK = 0x7fffffff;
constexpr int WAVE_CAP = 512;         // per-wavefront loser buffer (LDS entries)
constexpr int SUB = WAVES * WAVE_CAP; // worklist entries per LDS flush
constexpr int OVW = 32;               // overflow bitmap words per wavefront (colours 65..1088)
constexpr int TWAVE_MAX = 1024;       // largest degree handled by one wavefront
constexpr int BMW = 1024;             // workgroup bitmap words (32768 colours per window)

// Bucket b handles degrees (lo_b, hi_b]: 0:(0,8] 1:(8,16] 2:(16,32] 3:(32,t_wave] 4:(t_wave,inf)
__host__ __device__ inline int bucket_of(int deg, int twave) {
    return deg <= 8 ? 0 : deg <= 16 ? 1 : deg <= 32 ? 2 : deg <= twave ? 3 : 4;
}

// Device-resident control block.
struct Ctl {
    int cnt[2][8];      // worklist length per bucket, double-buffered by round parity
    int dyn[2][8];      // dynamic work counters for workgroup-per-vertex buckets (per phase)
    int hist[8];        // vertices per degree bucket (deg >= 1)
    int maxcolor;       // largest settled colour
    int err;            // bit 0: rowptr, bit 1: colidx range, bit 2: asymmetric, bit 3: internal
    int desc_total;     // positions e >= 1 with colidx[e] < colidx[e-1]
    int desc_bound;     // such positions that start a non-empty row
    int maxdeg;
    int rounds;         // number of non-empty rounds so far
    int nnz;            // rowptr[n]
    int pad;
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
    int sorted;         // 1: every row ascending -> conflict scans stop at the first w >= v
    int round;          // 0-based round index (round 0 is the round-1 shortcut)
    int st_cap;
    long long* st_wsize;
    long long* st_arcs;
    int seg[NB + 1];    // bucket segment offsets inside the worklist arrays
    int boff[NB + 1];   // block offsets of each bucket inside the grid
};

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
