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
    // grid barrier of the persistent round kernel
    unsigned int bar_count;
    unsigned int bar_gen;
    unsigned int pad0[2];
    // per-round ring: minimum priority, survivor count, packed frontier
    // counter (items << 38 | edges)
    unsigned int mn[4];
    unsigned int lcnt[4];
    unsigned long long fcnt[4];
    // results of the current iteration
    int nrounds;
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

// ------------------------------------------------------------ grid barrier
// Sense-reversing barrier over all blocks of a co-resident (cooperative)
// grid.  Release at agent scope before arriving, acquire after leaving, so
// plain stores made before the barrier by any block are visible to plain
// loads after it.
__device__ __forceinline__ void grid_barrier(Ctl* ctl, unsigned int nblocks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned int arrived =
            __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->bar_gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen)
                __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

}  // namespace dsg
