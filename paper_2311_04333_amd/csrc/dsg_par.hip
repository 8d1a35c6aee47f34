// dsg_par.hip -- kernels of the Pruning-and-Refining framework (Algorithm 1,
// Section 3 of Sukprasert, Liu, Dhulipala, Shun, arXiv 2311.04333) with
// exact k-core pruning: core numbers from a PEEL pass, and getCore (the
// subgraph induced by the vertices of core number >= j), built as scans and
// compactions so that a prune moves each adjacency entry once.
#include "dsg_device.h"
#include "dsg_par.h"

namespace dsg {

namespace {

constexpr int PBLK = 1024;
constexpr int PITEMS = 4;
constexpr int PTILE = PBLK * PITEMS;

inline int grid_cap(long long n, int blk, int cap) {
    long long g = (n + blk - 1) / blk;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// ------------------------------------------------------ exclusive scan
// out[0..N] = exclusive prefix sums of in[0..N) followed by the total.
// Three passes: per-tile sums, one block scanning the tile sums, per-tile
// scans with the tile offset.
__global__ __launch_bounds__(PBLK) void k_par_tilesum(const int* __restrict__ in, long long N,
                                                      long long* __restrict__ tiles) {
    __shared__ long long sh[PBLK / WAVE];
    const long long base = (long long)blockIdx.x * PTILE;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < PITEMS; k++) {
        const long long i = base + (long long)k * PBLK + threadIdx.x;
        if (i < N) s += in[i];
    }
    s = block_sum<PBLK>(s, sh);
    if (threadIdx.x == 0) tiles[blockIdx.x] = s;
}

__global__ __launch_bounds__(PBLK) void k_par_tiletop(long long* __restrict__ tiles, long long ntiles) {
    __shared__ long long sh[PBLK / WAVE];
    long long carry = 0;
    for (long long b = 0; b < ntiles; b += PBLK) {
        const long long i = b + threadIdx.x;
        const long long v = i < ntiles ? tiles[i] : 0;
        long long tot;
        const long long ex = block_excl_scan<PBLK>(v, &tot, sh);
        if (i < ntiles) tiles[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(PBLK) void k_par_scanapply(const int* __restrict__ in, long long N,
                                                        const long long* __restrict__ tiles, int* __restrict__ out) {
    __shared__ long long sh[PBLK / WAVE];
    const long long i0 = (long long)blockIdx.x * PTILE + (long long)threadIdx.x * PITEMS;
    int x[PITEMS];
    long long mine = 0;
#pragma unroll
    for (int k = 0; k < PITEMS; k++) {
        x[k] = i0 + k < N ? in[i0 + k] : 0;
        mine += x[k];
    }
    long long tot;
    long long run = tiles[blockIdx.x] + block_excl_scan<PBLK>(mine, &tot, sh);
#pragma unroll
    for (int k = 0; k < PITEMS; k++) {
        if (i0 + k < N) {
            out[i0 + k] = (int)run;
            run += x[k];
            if (i0 + k == N - 1) out[N] = (int)run;
        }
    }
}

__global__ void k_par_set(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

long long par_scan_tiles(long long count) { return (count + PTILE - 1) / PTILE + 1; }

static hipError_t exclusive_scan(const int* in, long long N, long long* tiles, int* out, hipStream_t s) {
    if (N <= 0) {
        k_par_set<<<1, 64, 0, s>>>(out, 0);
        return hipGetLastError();
    }
    const long long nt = (N + PTILE - 1) / PTILE;
    k_par_tilesum<<<(unsigned int)nt, PBLK, 0, s>>>(in, N, tiles);
    k_par_tiletop<<<1, PBLK, 0, s>>>(tiles, nt);
    k_par_scanapply<<<(unsigned int)nt, PBLK, 0, s>>>(in, N, tiles, out);
    return hipGetLastError();
}

// ------------------------------------------------------ core numbers
__global__ void k_par_fill(int* __restrict__ p, int v, long long cnt) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// rv[r] = max(rv[0..r]) in place; *kmax = rv[nrounds - 1] (0 without rounds)
__global__ __launch_bounds__(PBLK) void k_prefix_max(int* __restrict__ rv, int nrounds, int* __restrict__ kmax) {
    __shared__ int sh[PBLK];
    int carry = 0;
    for (int b = 0; b < nrounds; b += PBLK) {
        const int i = b + threadIdx.x;
        int v = i < nrounds ? rv[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        // inclusive max scan (Hillis-Steele) over the chunk
        for (int o = 1; o < PBLK; o <<= 1) {
            const int w = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] = max(sh[threadIdx.x], w);
            __syncthreads();
        }
        v = max(carry, sh[threadIdx.x]);
        if (i < nrounds) rv[i] = v;
        carry = max(carry, sh[PBLK - 1]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *kmax = carry;
}

__global__ void k_core_from_rounds(int n, int nrounds, const int* __restrict__ rnd, const int* __restrict__ rv,
                                   int* __restrict__ core) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int r = rnd[v];
        core[v] = (r >= 0 && r < nrounds) ? rv[r] : 0;
    }
}

hipError_t launch_core_numbers(const GraphDev& g, int nrounds, int* rv, int* core, int* kmax_dev, hipStream_t s) {
    k_prefix_max<<<1, PBLK, 0, s>>>(rv, nrounds, kmax_dev);
    k_core_from_rounds<<<grid_cap(g.n, 256, 2048), 256, 0, s>>>(g.n, nrounds, g.rnd, rv, core);
    return hipGetLastError();
}

// ------------------------------------------------------ getCore
__global__ void k_keep(int n, const int* __restrict__ oldid, const int* __restrict__ core, int level,
                       int* __restrict__ keep) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
        keep[x] = core[oldid[x]] >= level ? 1 : 0;
}

// f[e] = 1 when both endpoints of adjacency entry e are kept.  Edge-parallel
// over the static item list (every vertex with edges, in id order, so the
// concatenated edge index is the adjacency index): a block stages one
// chunk's items in LDS and each thread finds its entries' rows by binary
// search, so hub rows spread over many threads.
__global__ __launch_bounds__(SORT_BLK) void k_edge_keep(long long nnz, int K, const int* __restrict__ siv,
                                                        const int* __restrict__ sie, const int* __restrict__ scf,
                                                        const int* __restrict__ scl, const int* __restrict__ adj,
                                                        const int* __restrict__ keep, int* __restrict__ f) {
    __shared__ int fe[SORT_CH];
    __shared__ int vv[SORT_CH];
    const long long nchunks = (nnz + SORT_CH - 1) / SORT_CH;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long x0 = c * SORT_CH, x1 = min(nnz, x0 + SORT_CH);
        const int k0 = scf[c];
        const int k1 = (c + 1 < nchunks) ? scl[c] : K - 1;
        const int nitems = k1 - k0 + 1;
        if (nitems < 1 || nitems > SORT_CH) {
            // impossible for an item list built from checked offsets; mark
            // the chunk's entries dropped rather than index LDS out of range
            for (long long x = x0 + threadIdx.x; x < x1; x += SORT_BLK) f[x] = 0;
            continue;
        }
        for (int j = threadIdx.x; j < nitems; j += SORT_BLK) {
            fe[j] = sie[k0 + j];
            vv[j] = siv[k0 + j];
        }
        __syncthreads();
        for (long long x = x0 + threadIdx.x; x < x1; x += SORT_BLK) {
            int lo = 0, hi = nitems - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (fe[mid] <= x) lo = mid; else hi = mid - 1;
            }
            f[x] = (keep[vv[lo]] && keep[adj[x]]) ? 1 : 0;
        }
        __syncthreads();
    }
}

__global__ void k_compact_adj(long long nnz, const int* __restrict__ f, const int* __restrict__ fs,
                              const int* __restrict__ adj, const int* __restrict__ newid, int* __restrict__ new_adj) {
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < nnz; x += (long long)gridDim.x * blockDim.x)
        if (f[x]) new_adj[fs[x]] = newid[adj[x]];
}

__global__ void k_compact_rows(int n, long long nnz, const int* __restrict__ keep, const int* __restrict__ newid,
                               const int* __restrict__ off, const int* __restrict__ fs, const int* __restrict__ oldid,
                               const int* __restrict__ load, int* __restrict__ new_off, int* __restrict__ new_oldid,
                               int* __restrict__ new_load, long long* __restrict__ counts) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        if (keep[x]) {
            const int nx = newid[x];
            new_off[nx] = fs[off[x]];
            new_oldid[nx] = oldid[x];
            new_load[nx] = load[x];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int n_new = newid[n];
        const int nnz_new = fs[nnz];
        new_off[n_new] = nnz_new;
        counts[0] = n_new;
        counts[1] = nnz_new;
    }
}

hipError_t launch_get_core(const GraphDev& g, const CoreCut& c, hipStream_t s) {
    hipError_t e;
    k_keep<<<grid_cap(g.n, 256, 4096), 256, 0, s>>>(g.n, c.oldid, c.core, c.level, c.keep);
    if ((e = exclusive_scan(c.keep, g.n, c.tiles, c.newid, s)) != hipSuccess) return e;
    if (g.nnz > 0) {
        const long long nchunks = (g.nnz + SORT_CH - 1) / SORT_CH;
        k_edge_keep<<<(int)(nchunks < 8192 ? nchunks : 8192), SORT_BLK, 0, s>>>(g.nnz, g.n_items, g.siv, g.sie, g.scf,
                                                                                  g.scl, g.adj, c.keep, c.f);
    }
    if ((e = exclusive_scan(c.f, g.nnz, c.tiles, c.fs, s)) != hipSuccess) return e;
    if (g.nnz > 0)
        k_compact_adj<<<grid_cap(g.nnz, 256, 16384), 256, 0, s>>>(g.nnz, c.f, c.fs, g.adj, c.newid, c.new_adj);
    k_compact_rows<<<grid_cap(g.n, 256, 4096), 256, 0, s>>>(g.n, g.nnz, c.keep, c.newid, g.off, c.fs, c.oldid,
                                                             g.load, c.new_off, c.new_oldid, c.new_load, c.counts_dev);
    return hipGetLastError();
}

// ------------------------------------------------------ masks
__global__ void k_fill_u8(unsigned char* __restrict__ p, long long cnt) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_suffix_mask(int n, const int* __restrict__ order, const int* __restrict__ oldid, int idx,
                              unsigned char* __restrict__ mask) {
    for (int i = idx + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        mask[oldid[order[i]]] = 1;
}

__global__ void k_vertex_mask(int n, const int* __restrict__ oldid, unsigned char* __restrict__ mask) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) mask[oldid[x]] = 1;
}

hipError_t launch_suffix_mask(const GraphDev& g, const int* oldid, int idx, unsigned char* mask, long long n_input,
                              hipStream_t s) {
    k_fill_u8<<<grid_cap(n_input, 256, 4096), 256, 0, s>>>(mask, n_input);
    if (idx >= 0 && idx < g.n)
        k_suffix_mask<<<grid_cap(g.n - idx, 256, 4096), 256, 0, s>>>(g.n, g.order, oldid, idx, mask);
    return hipGetLastError();
}

hipError_t launch_vertex_mask(int n, const int* oldid, unsigned char* mask, long long n_input, hipStream_t s) {
    k_fill_u8<<<grid_cap(n_input, 256, 4096), 256, 0, s>>>(mask, n_input);
    if (n > 0) k_vertex_mask<<<grid_cap(n, 256, 4096), 256, 0, s>>>(n, oldid, mask);
    return hipGetLastError();
}

__global__ void k_iota(int* __restrict__ out, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = i;
}

hipError_t launch_iota(int* out, int n, hipStream_t s) {
    if (n > 0) k_iota<<<grid_cap(n, 256, 4096), 256, 0, s>>>(out, n);
    return hipGetLastError();
}

__global__ void k_scatter(const int* __restrict__ src, const int* __restrict__ idx, int n, int* __restrict__ dst) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) dst[idx[x]] = src[x];
}

hipError_t launch_scatter(const int* src, const int* idx, int n_src, int* dst, long long n_dst, hipStream_t s) {
    if (n_dst > 0) k_par_fill<<<grid_cap(n_dst, 256, 4096), 256, 0, s>>>(dst, 0, n_dst);
    if (n_src > 0) k_scatter<<<grid_cap(n_src, 256, 4096), 256, 0, s>>>(src, idx, n_src, dst);
    return hipGetLastError();
}

}  // namespace dsg
