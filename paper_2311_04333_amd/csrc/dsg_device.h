// dsg_device.h -- device-side building blocks for the Greedy++ peeling kernels
// (gfx950, wave64).  Internal to libdsg.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsg {

constexpr int WAVE = 64;

// Per-graph control block in device memory (inside the caller's workspace).
// Ring slots indexed by round & 3 hold per-round values; a slot is cleared
// two rounds ahead of its use, so no round reads a slot that another round
// is still writing.
struct alignas(256) Ctl {
    // per-round rings (slot = round mod 4), each counter array on its own
    // cache line: every block updates them with atomics
    alignas(128) unsigned int mn[4];          // minimum priority bid for the round
    alignas(128) unsigned int lcnt[4];        // survivor count
    alignas(128) unsigned long long fcnt[4];  // frontier items << 38 | frontier edges
    alignas(128) unsigned int cnext[4];       // next sweep chunk to hand out
    // near-list rounds only
    alignas(128) unsigned int pcnt[4];        // vertices peeled in the round
    alignas(128) unsigned int xcnt[4];        // entries of the round's crossing list
    alignas(128) unsigned int mn2[4];         // exact minimum of a round that rescans the full list first
    // results of the current iteration
    alignas(128) int nrounds;
    int improved;
    int iters_done;
    int best_iter;
    long long best_e;
    long long best_v;
    long long best_idx;
    // graph facts and checks
    int max_deg;
    int err_count;
    int err_code;
    int err_vertex;
    unsigned long long check_sum;
};

enum ErrCode {
    ERR_NONE = 0,
    ERR_OFF_FIRST = 1,
    ERR_OFF_LAST = 2,
    ERR_OFF_DECREASING = 3,
    ERR_ADJ_RANGE = 4,
    ERR_SELF_LOOP = 5,
    ERR_ROW_ORDER = 6,
    ERR_ASYMMETRIC = 7,
    ERR_INTERNAL = 8
};

// SplitMix64 output function of state z + golden gamma (the digest mixer).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------- wave ops
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, WAVE);
        v = w < v ? w : v;
    }
    return v;
}

// inclusive scan within the wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T w = __shfl_up(v, o, WAVE);
        if (lane >= o) v += w;
    }
    return v;
}

// Block-wide exclusive scan; returns the block total in *total.  `sh` must
// hold BLK/WAVE elements.  Contains __syncthreads().
template <int BLK, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* total, T* sh) {
    constexpr int NW = BLK / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    T inc = wave_incl_scan(v);
    if (lane == WAVE - 1) sh[wid] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        T s = sh[w];
        if (w < wid) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <int BLK, typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
    constexpr int NW = BLK / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) tot += sh[w];
    __syncthreads();
    return tot;
}

template <int BLK, typename T>
__device__ __forceinline__ T block_min(T v, T* sh) {
    constexpr int NW = BLK / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    v = wave_min(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    T m = sh[0];
#pragma unroll
    for (int w = 1; w < NW; w++) m = sh[w] < m ? sh[w] : m;
    __syncthreads();
    return m;
}

// Block barrier that orders LDS only: waits for this wave's LDS operations,
// then s_barrier.  Unlike __syncthreads it does not wait for outstanding
// global memory operations, so fire-and-forget global atomics stay in
// flight across it.  Use only where no global data written before it is
// read by another thread after it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ------------------------------------------------------------ grid barrier
// XCD (accelerator complex die) of the executing wave: hardware register
// XCC_ID, bits [2:0].  MI355X has 8 XCDs, each with its own L2.
__device__ __forceinline__ unsigned int xcd_id() {
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 0x7u;
}

// State of the XCD-grouped grid barrier; every field sits on its own cache
// line.  Zeroed before each launch of a kernel that uses it.
struct alignas(256) GridSync {
    unsigned int gen;
    unsigned int pad0[63];
    unsigned int started;
    unsigned int pad1[63];
    unsigned int gsize[8];
    unsigned int pad2[56];
    unsigned int gcnt;           // XCD releases (monotonic)
    unsigned int pad3[63];
    unsigned int xcnt[8][64];    // arrivals per XCD (monotonic)
};

__device__ __forceinline__ unsigned int ld_agent(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent_u64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned int* p, unsigned int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-block handle of the grid barrier.  Only thread 0 of a block runs the
// protocol, so only its copy of the counts is meaningful.
struct GridBarrier {
    GridSync* gs;
    unsigned int xid;    // this block's XCD
    unsigned int gsz;    // blocks of the launch on this XCD
    unsigned int nx;     // XCDs holding blocks of the launch
    unsigned int epoch;  // barriers passed in this launch
};

// Called once at kernel start by every block: count the blocks of each XCD
// in this launch (the block-to-XCD placement is the hardware's choice), wait
// until every block has counted, then keep the counts in registers.
__device__ __forceinline__ GridBarrier grid_sync_init(GridSync* gs, unsigned int nblocks, unsigned int xid) {
    GridBarrier b{gs, xid, 0u, 0u, 0u};
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&gs->gsize[xid], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&gs->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (ld_agent(&gs->started) < nblocks) __builtin_amdgcn_s_sleep(1);
        b.gsz = ld_agent(&gs->gsize[xid]);
        for (int x = 0; x < 8; x++) b.nx += ld_agent(&gs->gsize[x]) != 0u ? 1u : 0u;
    }
    __syncthreads();
    return b;
}

// Grid barrier with one L2 write-back per XCD instead of one per block
// (per-block agent-scope releases dominate the cost of a barrier at 256
// blocks).  Blocks of an XCD arrive on that XCD's counter after their own
// stores have completed into the shared L2.  The last arrival of an XCD
// issues the agent-scope release that writes that L2 back, waits for it,
// then arrives on the global counter; the arrival that completes the global
// count publishes the epoch.  Every block then performs its own agent-scope
// acquire (L1 and L2 invalidate, waited for).
//
// The barrier comes in two halves.  Between grid_arrive and grid_wait a
// block may read what was published at an earlier barrier and write LDS,
// but its global writes are not released by this barrier.
__device__ __forceinline__ void grid_arrive(GridBarrier& b) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    b.epoch++;
    if (threadIdx.x == 0) {
        GridSync* gs = b.gs;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned int a =
            __hip_atomic_fetch_add(&gs->xcnt[b.xid][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == b.epoch * b.gsz - 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            const unsigned int g =
                __hip_atomic_fetch_add(&gs->gcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (g == b.epoch * b.nx - 1) st_agent(&gs->gen, b.epoch);
        }
    }
}

__device__ __forceinline__ void grid_wait(GridBarrier& b) {
    if (threadIdx.x == 0) {
        while (ld_agent(&b.gs->gen) < b.epoch) __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
}

__device__ __forceinline__ void grid_sync(GridBarrier& b) {
    grid_arrive(b);
    grid_wait(b);
}

}  // namespace dsg
