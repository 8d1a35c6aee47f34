// dsg_kernels.hip -- HIP kernels for the Greedy++ peeling hot path on gfx950.
//
// Method: Sukprasert, Liu, Dhulipala, Shun, arXiv 2311.04333.
//   * ordering of one iteration:
//       SEQ  -- load ordering of Section 2, one vertex at a time (k_seq_order);
//       PEEL -- round-synchronous (1+eps)-of-minimum peeling, the parallel
//               ordering of Section 3.3 (k_peel_init + k_peel_rounds);
//       SORT -- sort by start-of-iteration load, Sections 3.2/3.3 (radix sort
//               + k_sort_pos + coarse classes k_coarse_tiles/bounds/pack
//               + k_sweep_sort);
//   * Algorithm 3 (density and load computation): each edge charges its
//     earlier endpoint (owner-computes sweep), suffix sums over positions, the
//     densest suffix as an exact rational, loads += charges (k_gather_A,
//     k_suffix_top, k_suffix_argmax, k_iter_end, k_finalize).
// All arithmetic is integer.  Device loads are int32; the host guarantees
// (iterations + 1) * max_degree < 2^31 so loads and priorities cannot wrap.
#include "dsg_device.h"
#include "dsg_internal.h"

namespace dsg {

// ================================================================ graph checks
// Offsets: off[0] == 0, off[n] == nnz, non-decreasing; also max degree.
__global__ void k_check_offsets(int n, long long nnz, const int* __restrict__ off, Ctl* ctl) {
    __shared__ int sh[WAVE];
    int local_max = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int a = off[v], b = off[v + 1];
        if (b < a) {
            if (atomicAdd(&ctl->err_count, 1) == 0) {
                ctl->err_code = ERR_OFF_DECREASING;
                ctl->err_vertex = v;
            }
        } else {
            local_max = max(local_max, b - a);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (off[0] != 0 && atomicAdd(&ctl->err_count, 1) == 0) {
            ctl->err_code = ERR_OFF_FIRST;
            ctl->err_vertex = 0;
        }
        if ((long long)off[n] != nnz && atomicAdd(&ctl->err_count, 1) == 0) {
            ctl->err_code = ERR_OFF_LAST;
            ctl->err_vertex = n;
        }
    }
    int lane = threadIdx.x & (WAVE - 1);
    for (int o = WAVE / 2; o > 0; o >>= 1) local_max = max(local_max, __shfl_xor(local_max, o, WAVE));
    if (lane == 0) atomicMax(&ctl->max_deg, local_max);
    (void)sh;
}

// Entries: every adj value in [0, n).  Runs only after the offsets passed.
__global__ void k_check_range(int n, long long nnz, const int* __restrict__ adj, Ctl* ctl) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (long long)gridDim.x * blockDim.x) {
        int u = adj[e];
        if (u < 0 || u >= n) {
            if (atomicAdd(&ctl->err_count, 1) == 0) {
                ctl->err_code = ERR_ADJ_RANGE;
                ctl->err_vertex = (int)(e & 0x7fffffff);
            }
        }
    }
}

// Full CSR check (DSG_VALIDATE): no self-loops, rows strictly increasing,
// symmetric (u in row v  =>  v in row u, by binary search in row u).
// Edge-parallel, so hub rows are spread over many threads, and it needs
// nothing but the (already checked) offsets: a block takes chunks of
// SORT_CH consecutive adjacency entries, finds the rows holding the chunk's
// first and last entry by binary search over all offsets, and each thread
// finds its entries' rows by binary search within that range (a few KB of
// offsets, cache-resident).  The row of entry x is the largest v with
// off[v] <= x: it skips empty rows, and off[v + 1] > x holds since
// off[n] = nnz > x.
__device__ __forceinline__ int row_of_entry(const int* __restrict__ off, int lo, int hi, long long x) {
    while (lo < hi) {
        const int mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(SORT_BLK) void k_check_rows(int n, long long nnz, const int* __restrict__ off,
                                                         const int* __restrict__ adj, Ctl* ctl) {
    __shared__ int s_k[2];
    const long long nchunks = (nnz + SORT_CH - 1) / SORT_CH;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long x0 = c * SORT_CH, x1 = min(nnz, x0 + SORT_CH);
        if (threadIdx.x < 2) s_k[threadIdx.x] = row_of_entry(off, 0, n - 1, threadIdx.x == 0 ? x0 : x1 - 1);
        __syncthreads();
        const int k0 = s_k[0], k1 = s_k[1];
        for (long long x = x0 + threadIdx.x; x < x1; x += SORT_BLK) {
            const int v = row_of_entry(off, k0, k1, x);
            const int u = adj[x];
            int code = ERR_NONE;
            if (u < 0 || u >= n) {  // callers may launch this before reading the range check's verdict
                code = ERR_ADJ_RANGE;
            } else if (u == v) {
                code = ERR_SELF_LOOP;
            } else if (x > off[v] && adj[x - 1] >= u) {
                code = ERR_ROW_ORDER;
            } else {
                int l = off[u], h = off[u + 1] - 1;
                bool found = false;
                while (l <= h) {
                    const int mid = l + ((h - l) >> 1);  // l + h can pass 2^31 when nnz > 2^30
                    const int w = adj[mid];
                    if (w == v) {
                        found = true;
                        break;
                    }
                    if (w < v) l = mid + 1; else h = mid - 1;
                }
                if (!found) code = ERR_ASYMMETRIC;
            }
            if (code != ERR_NONE && atomicAdd(&ctl->err_count, 1) == 0) {
                ctl->err_code = code;
                ctl->err_vertex = v;
            }
        }
        __syncthreads();  // s_k is rewritten for the next chunk
    }
}

__global__ void k_ctl_reset(Ctl* ctl, long long m, int n) {
    if (threadIdx.x == 0) {
        ctl->best_e = m;
        ctl->best_v = n;
        ctl->best_iter = 0;
        ctl->best_idx = 0;
        ctl->iters_done = 0;
        ctl->improved = 0;
        ctl->nrounds = 0;
    }
}

__global__ void k_fill_i32(int* __restrict__ p, int v, long long cnt) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ====================================================== generic tile scans
// Exclusive prefix sum of int32 counts over n entries, in three steps:
// per-tile sums, a one-block scan of the tile sums, per-tile scan + offset.
constexpr int SCAN_BLK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLK * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_BLK) void k_scan_tile_sums(const int* __restrict__ in, long long n,
                                                             long long* __restrict__ tile_sum) {
    __shared__ long long sh[SCAN_BLK / WAVE];
    long long base = (long long)blockIdx.x * SCAN_TILE;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k * SCAN_BLK + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = block_sum<SCAN_BLK>(s, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// One block: exclusive scan of tile sums in place; total into *total.
__global__ __launch_bounds__(1024) void k_scan_top(long long* __restrict__ tile_sum, int ntiles,
                                                   long long* __restrict__ total) {
    __shared__ long long sh[1024 / WAVE];
    long long carry = 0;
    for (int base = 0; base < ntiles; base += 1024) {
        int i = base + threadIdx.x;
        long long v = i < ntiles ? tile_sum[i] : 0;
        long long tot;
        long long ex = block_excl_scan<1024>(v, &tot, sh);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// ============================================================ radix sort
// Stable LSD radix sort of (key, value) int32 pairs by 8-bit digits.  Tile
// = 256 threads x 16 items.  Inside a tile, wave w owns the contiguous items
// [w*1024, (w+1)*1024) and walks them in 16 steps of 64 consecutive items.
// The stable rank among equal digits in a step comes from 8 ballots; the
// earlier steps of the wave and the earlier waves of the tile come from LDS
// counters; the earlier tiles come from the scanned digit-major histogram.
constexpr int RBLK = 256;
constexpr int RITEMS = 16;
constexpr int RTILE = RBLK * RITEMS;
constexpr int RBINS = 256;

// `gate` (optional): the pass is skipped when *gate <= 2^16, i.e. when every
// key is below 2^16 and the pass's digit is zero for all of them.
__device__ __forceinline__ bool radix_skip(const int* gate) { return gate && *gate <= (1 << 16); }

__global__ __launch_bounds__(RBLK) void k_radix_hist(const int* __restrict__ keys, int n, int shift,
                                                     int* __restrict__ hist, int ntiles, const int* gate) {
    if (radix_skip(gate)) return;
    __shared__ int h[RBINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * RTILE;
#pragma unroll
    for (int k = 0; k < RITEMS; k++) {
        int i = base + k * RBLK + threadIdx.x;
        if (i < n) atomicAdd(&h[((unsigned int)keys[i] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Digit-major exclusive scan of hist[RBINS * ntiles] in three kernels:
// per-tile sums, one-block scan of those sums, in-tile scan plus offset.
__global__ __launch_bounds__(SCAN_BLK) void k_rscan_tiles(const int* __restrict__ hist, int total,
                                                          long long* __restrict__ tile_sum, const int* gate) {
    if (radix_skip(gate)) return;
    __shared__ long long sh[SCAN_BLK / WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k;
        if (i < total) s += hist[i];
    }
    s = block_sum<SCAN_BLK>(s, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_rscan_top(long long* __restrict__ tile_sum, int ntiles, const int* gate) {
    if (radix_skip(gate)) return;
    __shared__ long long sh[1024 / WAVE];
    long long carry = 0;
    for (int base = 0; base < ntiles; base += 1024) {
        int i = base + threadIdx.x;
        long long v = i < ntiles ? tile_sum[i] : 0;
        long long tot;
        long long ex = block_excl_scan<1024>(v, &tot, sh);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_BLK) void k_rscan_apply(int* __restrict__ hist, int total,
                                                          const long long* __restrict__ tile_sum, const int* gate) {
    if (radix_skip(gate)) return;
    __shared__ long long sh[SCAN_BLK / WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    int x[SCAN_ITEMS];
    long long mine = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k;
        x[k] = i < total ? hist[i] : 0;
        mine += x[k];
    }
    long long tot;
    long long run = tile_sum[blockIdx.x] + block_excl_scan<SCAN_BLK>(mine, &tot, sh);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k;
        if (i < total) hist[i] = (int)run;
        run += x[k];
    }
}

// keys_in: key of item i; vals_in: value of item i (nullptr = i itself).
// keys_out may be nullptr (last pass).
__global__ __launch_bounds__(RBLK) void k_radix_scatter(const int* __restrict__ keys_in,
                                                        const int* __restrict__ vals_in, int* __restrict__ keys_out,
                                                        int* __restrict__ vals_out, int n, int shift,
                                                        const int* __restrict__ hist, int ntiles, const int* gate) {
    if (radix_skip(gate)) return;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    const int base = blockIdx.x * RTILE;
    __shared__ int wcnt[RBLK / WAVE][RBINS];
    __shared__ int tbase[RBINS];
    for (int d = tid; d < RBINS * (RBLK / WAVE); d += RBLK) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    int key[RITEMS], rank[RITEMS];
    const unsigned long long lower = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    const int wbase = base + wid * (WAVE * RITEMS);
#pragma unroll
    for (int s = 0; s < RITEMS; s++) {
        int i = wbase + s * WAVE + lane;
        bool ok = i < n;
        int k = ok ? keys_in[i] : 0;
        key[s] = k;
        unsigned int d = ((unsigned int)k >> shift) & 0xFF;
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            unsigned long long m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        int before = __popcll(peers & lower);
        int prev = ok ? wcnt[wid][d] : 0;
        rank[s] = prev + before;
        // all lanes of the wave have read the counter before any lane updates it
        __builtin_amdgcn_wave_barrier();
        if (ok && before == 0) wcnt[wid][d] = prev + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: global base of this tile + counts of earlier waves
    {
        int d = tid;  // RBLK == RBINS
        int run = hist[d * ntiles + blockIdx.x];
        tbase[d] = run;
#pragma unroll
        for (int w = 0; w < RBLK / WAVE; w++) {
            int c = wcnt[w][d];
            wcnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RITEMS; s++) {
        int i = wbase + s * WAVE + lane;
        if (i < n) {
            unsigned int d = ((unsigned int)key[s] >> shift) & 0xFF;
            int dst = wcnt[wid][d] + rank[s];
            if (keys_out) keys_out[dst] = key[s];
            vals_out[dst] = vals_in ? vals_in[i] : i;
        }
    }
    (void)tbase;
}

// Writes the chunk markers of one item occupying edges [start, end).
template <int CH>
__device__ __forceinline__ void mark_chunks(long long start, long long end, int item, int* __restrict__ cfirst,
                                            int* __restrict__ clast) {
    for (long long c = (start + CH - 1) / CH; c * CH < end; c++) cfirst[c] = item;
    // chunk c's last edge (c+1)*CH - 1 lies in [start, end)
    for (long long c = (start + 1 + CH - 1) / CH - 1; (c + 1) * CH <= end; c++) clast[c] = item;
}


// ============================================================ static items
// Items of the full graph for the SORT sweep: every vertex with degree > 0,
// in id order, with its edge start, row base and chunk markers.
__global__ void k_nonzero_flags(int n, const int* __restrict__ off, int* __restrict__ flag) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        flag[v] = off[v + 1] > off[v] ? 1 : 0;
}

__global__ __launch_bounds__(SCAN_BLK) void k_compact_items(int n, const int* __restrict__ off,
                                                            const long long* __restrict__ tile_off,
                                                            int* __restrict__ iv, int* __restrict__ ie,
                                                            int* __restrict__ ir, int* __restrict__ cfirst,
                                                            int* __restrict__ clast) {
    __shared__ int sh[SCAN_BLK / WAVE];
    long long base = (long long)blockIdx.x * SCAN_TILE;
    long long run = tile_off[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long v = base + k * SCAN_BLK + threadIdx.x;
        int a = 0, b = 0, f = 0;
        if (v < n) {
            a = off[v];
            b = off[v + 1];
            f = b > a;
        }
        int tot;
        int ex = block_excl_scan<SCAN_BLK>(f, &tot, sh);
        if (f) {
            int item = (int)(run + ex);
            iv[item] = (int)v;
            ie[item] = a;
            ir[item] = 0;  // the whole graph's rows are already concatenated in order
            mark_chunks<SORT_CH>(a, b, item, cfirst, clast);
        }
        run += tot;
    }
}

// ========================================================== edge sweep
// Edge-balanced sweep over the concatenated rows of an item list.  An item
// list holds, per item k: its vertex iv[k], its first edge ie[k] in the
// concatenation, and ir[k] = offsets[v] - ie[k], so edge x of the item is
// adj[ir[k] + x].  For every chunk c of CH consecutive edges it also holds
// cfirst[c] and clast[c], the items holding the chunk's first and last edge
// (clast of the final chunk is K - 1).  Block b takes chunks b, b + grid,
// and so on.  The chunk's items (at most CH, since each has an edge in the
// chunk) are staged in LDS.  Each thread handles EPT = CH / BLK edges.  It
// finds their items by binary search in LDS, issues all EPT adjacency loads,
// then all EPT neighbour-state gathers, then processes them.  That costs
// two memory round trips per chunk instead of two per edge.  Per-item
// counts are gathered in LDS and added to inc[] once per chunk.
template <int CH>
struct SweepLds {
    int fe[CH];
    int rb[CH];
    int v[CH];
    int cnt[CH];
};

// Chunks are handed out by an atomic counter (`cnext`, zero at the start)
// when it is given, else statically (b, b + grid, ...).  The block
// barriers inside a chunk order LDS only, so the chunk's global atomics
// (charges, aggregated decrements) overlap the next chunk's loads.  The
// markers may be finer than the chunk: MS markers per chunk, so chunk c
// starts at item cfirst[c * MS] and ends at item clast[c * MS + MS - 1].
// With PF > 0 (dynamic chunks only), the first PF * BLK items of the block's
// next chunk, and its item range, are loaded into registers while the current
// chunk is processed, which takes two dependent memory round trips (markers,
// then items) off the start of every chunk.
template <int BLK, int CH, int MS, class Op, class Lds, int PF = 0>
__device__ __forceinline__ void sweep_chunks(int K, long long E, const int* __restrict__ iv, const int* __restrict__ ie,
                                             const int* __restrict__ ir, const int* __restrict__ cfirst,
                                             const int* __restrict__ clast, const int* __restrict__ adj,
                                             int* __restrict__ inc, Op& op, Lds& s, int block, int nblocks,
                                             unsigned int* cnext, int* s_chunk) {
    constexpr int EPT = CH / BLK;
    static_assert(EPT * BLK == CH, "chunk must be a multiple of the block");
    static_assert(sizeof(s.fe) >= sizeof(int) * CH, "LDS item arrays must hold a chunk's items");
    const long long nchunks = (E + CH - 1) / CH;
    long long c = block;
    if (cnext) {
        if (threadIdx.x == 0) *s_chunk = (int)atomicAdd(cnext, 1u);
        lds_barrier();
        c = *s_chunk;
        lds_barrier();
    }
    // item range of chunk cc: [k0, k1]
    auto range = [&](long long cc, int& k0, int& k1) {
        k0 = cfirst[cc * MS];
        k1 = (cc + 1 < nchunks) ? clast[cc * MS + MS - 1] : K - 1;
    };
    int pk0 = 0, pk1 = -1;       // prefetched chunk's item range (valid when pf_ok)
    bool pf_ok = false;
    int pv[PF > 0 ? PF : 1], pe[PF > 0 ? PF : 1], pr[PF > 0 ? PF : 1];
    for (; c < nchunks;) {
        const long long x0 = c * CH;
        const long long x1 = min(E, x0 + CH);
        int k0, k1;
        if (PF > 0 && pf_ok) {
            k0 = pk0;
            k1 = pk1;
        } else {
            range(c, k0, k1);
        }
        const int nitems = k1 - k0 + 1;
        if (nitems < 1 || nitems > CH) {
            // impossible when every item has an edge in the chunk; refuse to
            // index LDS out of range if the item list is ever inconsistent
            if (threadIdx.x == 0) op.flag_error();
            break;
        }
        // grab the next chunk while this one is processed
        if (cnext && threadIdx.x == 0) *s_chunk = (int)atomicAdd(cnext, 1u);
        int jstart = 0;
        if (PF > 0 && pf_ok) {
#pragma unroll
            for (int q = 0; q < (PF > 0 ? PF : 1); q++) {
                const int j = (int)threadIdx.x + q * BLK;
                if (j < nitems) {
                    s.fe[j] = pe[q];
                    s.rb[j] = pr[q];
                    s.v[j] = pv[q];
                    s.cnt[j] = 0;
                    op.stage_item(j, pv[q]);
                }
            }
            jstart = (PF > 0 ? PF : 1) * BLK;
        }
        for (int j = jstart + (int)threadIdx.x; j < nitems; j += BLK) {
            const int v = iv[k0 + j];
            s.fe[j] = ie[k0 + j];
            s.rb[j] = ir[k0 + j];
            s.v[j] = v;
            s.cnt[j] = 0;
            op.stage_item(j, v);
        }
        lds_barrier();
        // the next chunk's id is in LDS since the barrier: start loading its
        // item range now (the items themselves follow the adjacency loads)
        long long cn = nchunks;
        if (PF > 0 && cnext) {
            cn = *s_chunk;
            pf_ok = cn < nchunks;
            if (pf_ok) range(cn, pk0, pk1);
        }
        // thread t owns the EPT consecutive edges from x0 + t*EPT: one binary
        // search for the first, then a linear advance over item boundaries
        const int xs = (int)x0 + (int)threadIdx.x * EPT;
        int jj[EPT], uu[EPT], st[EPT];
        unsigned int tl = 0;  // bit e: entry e's order flag (bit 31 of a renumbered CSR's entry)
        {
            int j = 0;
            if ((long long)xs < x1) {
                int hi = nitems - 1;
                while (j < hi) {
                    int mid = (j + hi + 1) >> 1;
                    if (s.fe[mid] <= xs) j = mid; else hi = mid - 1;
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; e++) {
                const int x = xs + e;
                if ((long long)x < x1) {
                    while (j + 1 < nitems && s.fe[j + 1] <= x) j++;
                    jj[e] = j;
                    const int raw = adj[s.rb[j] + x];
                    uu[e] = raw & ADJ_ID_MASK;
                    tl |= (raw < 0 ? 1u : 0u) << e;
                } else {
                    jj[e] = -1;
                    uu[e] = 0;
                }
            }
        }
        if (PF > 0 && pf_ok) {
            const int nn = pk1 - pk0 + 1;
#pragma unroll
            for (int q = 0; q < (PF > 0 ? PF : 1); q++) {
                const int j = (int)threadIdx.x + q * BLK;
                const bool in = j < nn && nn <= CH;
                pv[q] = in ? iv[pk0 + j] : 0;
                pe[q] = in ? ie[pk0 + j] : 0;
                pr[q] = in ? ir[pk0 + j] : 0;
            }
        }
        (void)cn;
#pragma unroll
        for (int e = 0; e < EPT; e++) st[e] = jj[e] >= 0 ? op.gather(uu[e]) : 0;
        op.template resolve<EPT>(jj, uu, st);
        bool hit[EPT];
#pragma unroll
        for (int e = 0; e < EPT; e++) hit[e] = jj[e] >= 0 && op.edge(s.v[jj[e]], uu[e], st[e], jj[e], (tl >> e) & 1u);
        // Per-item counts.  Same-address LDS atomics serialise, and in a hub
        // row every edge of the chunk has the same item, so the counts are
        // summed first: over runs of one item within the thread's consecutive
        // edges, then over the wave when all its lanes end on one item.
        int rj = jj[0], rc = 0;
#pragma unroll
        for (int e = 0; e < EPT; e++) {
            if (jj[e] != rj) {
                if (rc) atomicAdd(&s.cnt[rj], rc);
                rj = jj[e];
                rc = 0;
            }
            rc += hit[e] ? 1 : 0;
        }
        const int j0 = __builtin_amdgcn_readfirstlane(rj);
        if (__all(rj == j0)) {
            const int tot = wave_sum(rc);
            if ((threadIdx.x & (WAVE - 1)) == 0 && tot) atomicAdd(&s.cnt[j0], tot);
        } else if (rc) {
            atomicAdd(&s.cnt[rj], rc);
        }
        lds_barrier();
        for (int j = threadIdx.x; j < nitems; j += BLK)
            if (s.cnt[j]) atomicAdd(&inc[s.v[j]], s.cnt[j]);
        op.flush_chunk();
        lds_barrier();
        if (cnext) {
            c = *s_chunk;
            lds_barrier();
        } else {
            c += nblocks;
        }
    }
}

// ============================================================== PEEL
// Iteration start: prio = load + degree, round = -1 (alive), charge = 0;
// the minimum priority seeds round 0.
__global__ __launch_bounds__(256) void k_peel_init(int n, const int* __restrict__ off, const int* __restrict__ load,
                                                   int* __restrict__ prio, int* __restrict__ rnd,
                                                   int* __restrict__ inc, unsigned int* __restrict__ st2, Ctl* ctl) {
    __shared__ unsigned int sh[256 / WAVE];
    unsigned int lmin = 0xFFFFFFFFu;
    // 2-bit state per vertex, 16 per word: every vertex alive (01), none in
    // a frontier
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < (n + 15) / 16; w += gridDim.x * blockDim.x)
        st2[w] = 0x55555555u;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int p = load[v] + (off[v + 1] - off[v]);
        prio[v] = p;
        rnd[v] = -1;
        inc[v] = 0;
        lmin = min(lmin, (unsigned int)p);
    }
    lmin = block_min<256>(lmin, sh);
    if (threadIdx.x == 0) atomicMin(&ctl->mn[0], lmin);
}

// Clears the per-iteration control fields, the grid-barrier state and the
// owner-bucket fill counters.
__global__ void k_iter_begin(Ctl* ctl, GridSync* gs, unsigned int* bfill, int nr) {
    for (int j = threadIdx.x; j < nr; j += blockDim.x) bfill[j] = 0;
    if (threadIdx.x < 4) {
        ctl->mn[threadIdx.x] = 0xFFFFFFFFu;
        ctl->lcnt[threadIdx.x] = 0;
        ctl->fcnt[threadIdx.x] = 0;
        ctl->cnext[threadIdx.x] = 0;
        ctl->pcnt[threadIdx.x] = 0;
        ctl->xcnt[threadIdx.x] = 0;
        ctl->mn2[threadIdx.x] = 0xFFFFFFFFu;
    }
    if (threadIdx.x == 0) {
        ctl->nrounds = 0;
        ctl->improved = 0;
    }
    if (gs) {
        unsigned int* w = reinterpret_cast<unsigned int*>(gs);
        for (unsigned int i = threadIdx.x; i < sizeof(GridSync) / 4; i += blockDim.x) w[i] = 0;
    }
}

// Open-addressing LDS table that aggregates degree decrements per target
// vertex within one chunk.  A hub adjacent to many of the chunk's edges then
// receives one global atomic instead of one per edge (same-address atomics
// serialise at about 11 ns each).  Probing is bounded; a target that finds
// no slot within PROBE steps is decremented directly in global memory.
constexpr int DEC_SLOTS = 2 * PEEL_CH;  // at most PEEL_CH keys: probing always finds a slot
constexpr int XS_CAP = BKT_MAX_NR;       // crossing staging entries (in the bucket flush's base array)
constexpr int DEC_PROBE = 64;
constexpr int DEC_EMPTY = -1;

struct DecTable {
    int key[DEC_SLOTS];
    int cnt[DEC_SLOTS];
};

struct PeelSweepLds {
    SweepLds<PEEL_CH> sw;
    DecTable dec;
};
// The bucket apply's per-range histogram in LDS.  Wide: one int counter per
// local id (2^15 ids).  Narrow (hub order when every vertex past the hub ids
// has degree below 2^16, so no count of one round reaches 2^16): 16-bit
// counters, two per int, for 2^16 local ids, and the range's first nh local
// ids (the hubs, of any degree) in ints of their own.  Halving the ranges
// halves the apply's per-range round trips and the flush's reservations.
struct DenseHist {
    int* d;    // 2^BKT_MAX_SHIFT ints
    int* hub;  // nh ints (narrow)
    int nh;
    bool narrow;
    unsigned int limit;  // local ids below this have a counter
    __device__ __forceinline__ void clear(int tid, int blk) const {
        for (int i = tid; i < (narrow ? (1 << BKT_MAX_SHIFT) : (int)limit); i += blk) d[i] = 0;
        if (narrow)
            for (int i = tid; i < nh; i += blk) hub[i] = 0;
    }
    __device__ __forceinline__ void add(unsigned int li, int c) const {
        if (li >= limit) return;
        if (!narrow) {
            atomicAdd(&d[li], c);
        } else if ((int)li < nh) {
            atomicAdd(&hub[li], c);
        } else {
            const unsigned int k = li - (unsigned int)nh;
            atomicAdd(&d[k >> 1], c << ((k & 1u) * 16));
        }
    }
    // the count of local id li (< limit), cleared
    __device__ __forceinline__ int take(unsigned int li) const {
        if (!narrow) return atomicExch(&d[li], 0);
        if ((int)li < nh) return atomicExch(&hub[li], 0);
        const unsigned int k = li - (unsigned int)nh;
        const int sh = (int)(k & 1u) * 16;
        const int old = atomicAnd(&d[k >> 1], ~(0xFFFF << sh));
        return (old >> sh) & 0xFFFF;
    }
};

struct PeelLds {
    union {
        PeelSweepLds m;                     // the sweep
        int dense[1 << BKT_MAX_SHIFT];      // the bucketed apply step (after the sweep)
    };
    int bcnt[BKT_MAX_NR];   // per-range entries of the chunk being flushed
    int bbase[BKT_MAX_NR];  // their reserved start in the range's bucket
    int spref[PEEL_BLK];    // select: virtual start of each block's segment of the alive list
    int sstart[PEEL_BLK];   // ... and its physical start
};
static_assert(sizeof(PeelSweepLds) >= sizeof(int) * (1 << BKT_MAX_SHIFT), "dense histogram aliases the sweep");

// What an edge (v, u) of a frontier vertex v does in round r:
//   u alive after the round (round[u] == -1): v is charged the edge, and
//     u loses one degree (aggregated per chunk in LDS, then one atomicSub
//     per distinct u); u's new priority bids for the next round's minimum.
//     Its last decrement yields its final value.
//   u peeled in the same round: the edge goes to the lower id.
//   u peeled earlier: nothing.
// Vertex state during a round, 2 bits per vertex packed 16 to a word (so the
// state of a 4M-vertex graph is 1 MB and stays in each XCD's L2 during the
// sweep): bit 0 = not peeled before this round, bit 1 = in this round's
// frontier.  01 = survives the round, 11 = peeled this round, 00 = peeled
// earlier.
__device__ __forceinline__ int st2_get(const unsigned int* st2, int u) {
    return (int)((st2[u >> 4] >> ((u & 15) * 2)) & 3u);
}

// Crossing list staging for one block: entries go to an LDS buffer with one
// LDS atomic per wave, and the buffer goes to the global list with one global
// atomic per flush (one global counter shared by every block serialises at
// about 11 ns per atomic).  Lanes that find the buffer full append directly.
struct XStage {
    int* xs;              // LDS buffer of XS_CAP entries
    unsigned int* xn;     // LDS count (may pass XS_CAP: the excess went to the global list directly)
    int* xout;            // global list
    unsigned int* xcnt;   // its count
    int cap;              // global capacity (n)
    Ctl* ctl;
    __device__ __forceinline__ void direct(int u) const {
        const unsigned int at = atomicAdd(xcnt, 1u);
        if (at < (unsigned int)cap) {
            xout[at] = u;
        } else {
            atomicAdd(&ctl->err_count, 1);
            ctl->err_code = ERR_INTERNAL;
        }
    }
    // every lane of the wave calls it
    __device__ __forceinline__ void stage_wave(bool x, int u) const {
        const unsigned long long m = __ballot(x);
        if (m == 0ull) return;
        const int lane = (int)(threadIdx.x & (WAVE - 1));
        const int leader = __ffsll((long long)m) - 1;
        unsigned int base = 0;
        if (lane == leader) base = atomicAdd(xn, (unsigned int)__popcll(m));
        base = (unsigned int)__shfl((int)base, leader, WAVE);
        if (x) {
            const unsigned int at = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
            if (at < (unsigned int)XS_CAP) xs[at] = u; else direct(u);
        }
    }
    // Block-uniform call point; `sbase` is an LDS word.  Leaves the buffer empty.
    __device__ __forceinline__ void flush(unsigned int* sbase) const {
        __syncthreads();
        const unsigned int k = min(*xn, (unsigned int)XS_CAP);
        if (k == 0u) return;  // uniform: every thread read the same count after the barrier
        if (threadIdx.x == 0) *sbase = atomicAdd(xcnt, k);
        __syncthreads();
        const unsigned int b = *sbase;
        for (unsigned int i = threadIdx.x; i < k; i += blockDim.x) {
            if (b + i < (unsigned int)cap) {
                xout[b + i] = xs[i];
            } else if (i == threadIdx.x) {
                atomicAdd(&ctl->err_count, 1);
                ctl->err_code = ERR_INTERNAL;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) *xn = 0u;
        __syncthreads();
    }
};

template <int BLK>
struct PeelEdgeOp {
    const unsigned int* st2;
    int* prio;
    int r;
    unsigned int lmin;
    Ctl* ctl;
    DecTable* dec;
    // bucketed rounds: the chunk's aggregated (target, count) pairs go to
    // the owner range's bucket instead of one atomicSub per target
    bool bucket;
    BktMap bm;
    int nr;
    int n;
    const int* rbase;
    int* bkt;
    unsigned int* bfill;
    int* bcnt;
    int* bbase;
    // near-list rounds: a decrement that takes a priority from above nearB to
    // at or below it appends the vertex to the next round's crossing list
    int nearB = -1;  // -1: off
    XStage xst{};
    // hub order: the entry's flag, not the internal ids, says which of two
    // vertices peeled in one round comes first (the smaller caller id)
    bool hub = false;
    __device__ void flag_error() {
        atomicAdd(&ctl->err_count, 1);
        ctl->err_code = ERR_INTERNAL;
    }
    __device__ __forceinline__ void stage_item(int, int) {}
    __device__ __forceinline__ int gather(int u) const { return st2_get(st2, u); }
    template <int EPT>
    __device__ __forceinline__ void resolve(const int (&)[EPT], const int (&)[EPT], int (&)[EPT]) const {}
    __device__ __forceinline__ bool edge(int v, int u, int su, int, unsigned int later_id) {
        if (su == 1) {
            unsigned int h = ((unsigned int)u * 0x9E3779B1u) >> (32 - __builtin_ctz(DEC_SLOTS));
#pragma unroll 1
            for (int probe = 0; probe < DEC_PROBE; probe++) {
                const int k = atomicCAS(&dec->key[h], DEC_EMPTY, u);
                if (k == DEC_EMPTY || k == u) {
                    atomicAdd(&dec->cnt[h], 1);
                    return true;
                }
                h = (h + 1) & (DEC_SLOTS - 1);
            }
            const int old = atomicSub(&prio[u], 1);
            lmin = min(lmin, (unsigned int)(old - 1));
            // (directly to the global list: in bucketed rounds the staging
            // buffer is the bucket flush's scratch)
            if (nearB >= 0 && old > nearB && old - 1 <= nearB) xst.direct(u);
            return true;
        }
        return su == 3 && (hub ? later_id != 0u : u > v);
    }
    __device__ __forceinline__ void flush_chunk() {
        if (bucket) {
            flush_to_buckets();
            return;
        }
        constexpr int PER = DEC_SLOTS / BLK;
        static_assert(PER * BLK == DEC_SLOTS, "slots must be a multiple of the block");
        lds_barrier();
        int key[PER], c[PER], old[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int slot = threadIdx.x + k * BLK;
            key[k] = dec->key[slot];
            c[k] = dec->cnt[slot];
        }
#pragma unroll
        for (int k = 0; k < PER; k++)
            if (key[k] != DEC_EMPTY) old[k] = atomicSub(&prio[key[k]], c[k]);
#pragma unroll
        for (int k = 0; k < PER; k++) {
            if (key[k] != DEC_EMPTY) {
                lmin = min(lmin, (unsigned int)(old[k] - c[k]));
                const int slot = threadIdx.x + k * BLK;
                dec->key[slot] = DEC_EMPTY;
                dec->cnt[slot] = 0;
            }
        }
        if (nearB >= 0) {
#pragma unroll
            for (int k = 0; k < PER; k++)
                xst.stage_wave(key[k] != DEC_EMPTY && old[k] > nearB && old[k] - c[k] <= nearB, key[k]);
        }
    }
    // Ranks each aggregated target within its owner range (LDS counters),
    // reserves the chunk's share of every touched range's bucket with one
    // global atomic per range, then writes the entries.  A range's bucket
    // holds at most one entry per decrement of its vertices in a round, so
    // its capacity is the range's degree sum: rbase[j + 1] - rbase[j].
    __device__ __forceinline__ void flush_to_buckets() {
        constexpr int PER = DEC_SLOTS / BLK;
        lds_barrier();
        int key[PER], c[PER], rk[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int slot = threadIdx.x + k * BLK;
            key[k] = dec->key[slot];
            c[k] = dec->cnt[slot];
            rk[k] = key[k] != DEC_EMPTY ? atomicAdd(&bcnt[bm.owner(key[k])], 1) : 0;
        }
        lds_barrier();
        for (int j = threadIdx.x; j < nr; j += BLK) {
            const int cj = bcnt[j];
            if (cj) {
                const int lo = rbase[j];
                const int hi = rbase[j + 1];
                const int b = lo + (int)atomicAdd(&bfill[j], (unsigned int)cj);
                if (b + cj > hi) {  // impossible by the capacity argument; never write past the range
                    flag_error();
                    bbase[j] = -1;
                } else {
                    bbase[j] = b;
                }
                bcnt[j] = 0;
            }
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            if (key[k] != DEC_EMPTY) {
                const int j = bm.owner(key[k]);
                const int b = bbase[j];
                if (b >= 0) bkt[b + rk[k]] = (bm.local(key[k]) << BKT_CNT_BITS) | (c[k] - 1);
                const int slot = threadIdx.x + k * BLK;
                dec->key[slot] = DEC_EMPTY;
                dec->cnt[slot] = 0;
            }
        }
    }
};

// Under hub order, the order in which the first full-list pass of an
// iteration visits the vertices (and so the order of the full list after it):
// 32-id lines read column by column from a 256-column row-major layout of the
// lines.  Every block's slice then samples the whole id space, so the blocks
// share the frontier evenly although vertices of similar degree, which tend
// to leave in the same rounds, have neighbouring ids.  A bijection of [0, n);
// the partial last line stays in place.
__device__ __forceinline__ int spread_id(int idx, int n) {
    constexpr int S = 256;
    const int nl = n >> 5;
    const int line = idx >> 5;
    if (line >= nl) return idx;
    const int rows = (nl + S - 1) / S;
    const int cfull = nl - (rows - 1) * S;  // columns with `rows` lines
    int col, row;
    if (line < cfull * rows) {
        col = line / rows;
        row = line - col * rows;
    } else {
        const int p = line - cfull * rows;
        col = cfull + p / (rows - 1);
        row = p - (col - cfull) * (rows - 1);
    }
    return ((row * S + col) << 5) | (idx & 31);
}

constexpr unsigned long long FCNT_SHIFT = 38;
constexpr unsigned long long FCNT_MASK = (1ull << FCNT_SHIFT) - 1;
// Alive-list entries per thread per select tile.  The round kernel is
// register-bound (128 VGPRs at 1024 threads): at 2 the select's arrays leave
// no VGPR spills, and the whole loop runs 7.5% faster than at 4 (25 spilled
// VGPRs) on R-MAT scale 22; at 8 (56 spilled) it is 35% slower.
constexpr int SEL_U = 2;
// Packed per-tile item scan value: [edges: bits 0-31][items: 45-63]; the
// select's per-tile survivor and item counts share a 32-bit word (16 bits
// each), and its frontier count is the tile's entries less its survivors.
constexpr int TITEM_SHIFT = 45;
static_assert(PEEL_BLK * SEL_U < (1 << 16), "tile counts must fit their packed fields");

// Persistent round loop of one PEEL iteration (cooperative launch, one block
// per CU).  Per round r:
//   select: mn = ring.mn[r]; thr = floor((q + p) mn / q) (MONO: at least the
//     previous round's thr).  Block b owns a contiguous slice of the alive
//     list L_r.  One pass classifies it: alive vertices with prio <= thr form
//     the frontier and are marked round r; the others survive.  Survivors go
//     to the head of the block's own segment of L_{r+1}, frontier vertices to
//     its tail, with no global reservation.  The frontier vertices with edges
//     then go to the item list (vertex, edge start, row base, chunk markers)
//     at a range reserved by one packed 64-bit atomic holding their count and
//     edge total, so item order and edge offsets agree.  Survivors bid their
//     priority for ring.mn[r+1].
//   grid sync
//   sweep: edge-balanced over the round's items (PeelEdgeOp).  In rounds
//     with many frontier edges the aggregated decrements go to owner-range
//     buckets, and after one more grid sync each block applies its ranges'
//     buckets (global atomics run at about 27 G/s on random targets, which
//     bounded those rounds).
//   grid sync, in two halves: between them each block builds its map of
//     L_{r+1} from the segment table and copies its frontier to the order
//     (positions by round, ascending id inside a round).
// L_0 is implicit (all vertices).  The loop ends when L_r is empty.  Every
// block reads the same counters after a grid sync, so all leave together.
// HUB: the graph is hub-ordered (a.hub), as a template argument so that the
// caller-order instantiation carries none of its registers.
template <bool MONO, bool HUB>
__global__ __launch_bounds__(PEEL_BLK, PEEL_BLOCKS_PER_CU) void k_peel_rounds(PeelArgs a) {
    __shared__ PeelLds lds;
    __shared__ int s_hubh[BKT_HUB_IDS >> BKT_NARROW_MIN_SB];  // narrow apply: the hubs' counters
    __shared__ unsigned long long shs[PEEL_BLK / WAVE];
    __shared__ unsigned int shm[PEEL_BLK / WAVE];
    __shared__ unsigned long long s_fbase;
    __shared__ int s_chunk;
    __shared__ long long s_thr;  // previous round's threshold (MONO)
    __shared__ unsigned long long s_segtot;  // entries in the previous round's segments
    Ctl* ctl = a.ctl;
    GridSync* gs = a.gs;
    const unsigned int nblocks = gridDim.x;
    const long long q = a.eps_den, p = a.eps_num;
    for (int slot = threadIdx.x; slot < DEC_SLOTS; slot += PEEL_BLK) {
        lds.m.dec.key[slot] = DEC_EMPTY;
        lds.m.dec.cnt[slot] = 0;
    }
    for (int j = threadIdx.x; j < BKT_MAX_NR; j += PEEL_BLK) lds.bcnt[j] = 0;
    GridBarrier bar = grid_sync_init(gs, nblocks, xcd_id());
    int prevLc = a.n + 1;
    for (int r = 0;; r++) {
        const int slot = r & 3, nslot = (r + 1) & 3;
        const unsigned int mn = ld_agent(&ctl->mn[slot]);
        const int Lc = (r == 0) ? a.n : (int)ld_agent(&ctl->lcnt[slot]);
        if (Lc == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) ctl->nrounds = r;
            break;
        }
        if (Lc >= prevLc) {
            // every round peels the minimum vertex, so the alive count must
            // fall; all blocks see the same counts and leave together
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ctl->nrounds = r;
                atomicAdd(&ctl->err_count, 1);
                ctl->err_code = ERR_INTERNAL;
            }
            break;
        }
        prevLc = Lc;
        long long thr = ((q + p) * (long long)mn) / q;
        if constexpr (MONO) {
            // Coreness by buckets: peel everything at or below the largest
            // threshold so far (the round's vertices all have core number thr)
            if (r > 0) thr = max(thr, s_thr);
            __syncthreads();
            if (threadIdx.x == 0) s_thr = thr;
        }
        // the round's bound (with zero loads and eps = 0 it is the core number
        // of every vertex the round peels; with eps > 0 an approximate one)
        if (a.rmin && blockIdx.x == 0 && threadIdx.x == 0) a.rmin[r] = (int)min(thr, 0x7FFFFFFFLL);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int zs = (r + 2) & 3;
            ctl->mn[zs] = 0xFFFFFFFFu;
            ctl->lcnt[zs] = 0;
            ctl->fcnt[zs] = 0;
            ctl->cnext[zs] = 0;
        }
        const int* __restrict__ Lin = (r & 1) ? a.L1 : a.L0;
        int* __restrict__ Lout = (r & 1) ? a.L0 : a.L1;
        int* __restrict__ ivr = (r & 1) ? a.iv1 : a.iv0;  // this round's item vertices
        if (r > 0) {
            // the previous round's frontier is peeled now: clear its state
            // bits (its vertices with edges are exactly its item list; the
            // isolated ones are never looked up)
            const int* __restrict__ ivp = (r & 1) ? a.iv0 : a.iv1;
            const int Kp = (int)(ld_agent_u64(&ctl->fcnt[(r - 1) & 3]) >> FCNT_SHIFT);
            for (int k = blockIdx.x * PEEL_BLK + threadIdx.x; k < Kp; k += nblocks * PEEL_BLK) {
                const int u = ivp[k];
                atomicAnd(&a.st2[u >> 4], ~(3u << ((u & 15) * 2)));
            }
        }
        // ---------------- select: this block's slice [beg, end) of L_r, in
        // tiles of PEEL_BLK * SEL_U entries; thread t owns SEL_U consecutive
        // entries.  L_r is virtual: the concatenation, in block order, of the
        // segments the blocks wrote in round r - 1 (segment j starts at
        // seg[start][j] of Lin and holds seg[len][j] entries); L_0 is all
        // vertices.  Block b writes its survivors to Lout[beg, beg + S) and
        // its frontier vertices to the tail Lout[end - F, end) (in reverse),
        // both in one pass without any global reservation, so only the
        // frontier is read again: to place the ones with edges in the item
        // list, and to write all of them to the order.
        const int per = (Lc + (int)nblocks - 1) / (int)nblocks;
        const int beg = min(Lc, (int)blockIdx.x * per), end = min(Lc, beg + per);
        constexpr int TILE = PEEL_BLK * SEL_U;
        unsigned int lmin = 0xFFFFFFFFu;
        unsigned long long my_edges = 0;
        int* __restrict__ seg_out = a.seg + (r & 1) * 3 * PEEL_BLK;  // [start | len | frontier len]
        // lds.spref / lds.sstart / s_segtot were filled from the previous
        // round's table inside the round-end barrier.  The segments hold
        // exactly the alive count (both are sums of the same per-block
        // survivor counts); never map past them.
        const bool map_ok = r == 0 || s_segtot == (unsigned long long)Lc;
        if (!map_ok && blockIdx.x == 0 && threadIdx.x == 0) {
            atomicAdd(&ctl->err_count, 1);
            ctl->err_code = ERR_INTERNAL;
        }
        // physical position in Lin of virtual index idx < Lc (r > 0): the last
        // segment whose prefix is <= idx holds it (empty ones are skipped).
        // A thread's indices only grow, so it finds its first segment by
        // binary search and then walks forward (usually not at all).
        int sj = 0;
        if (r > 0 && map_ok) {
            const int first = beg + (int)threadIdx.x * SEL_U;
            int lo = 0, hi = (int)nblocks - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (lds.spref[mid] <= first) lo = mid; else hi = mid - 1;
            }
            sj = lo;
        }
        auto phys = [&](int idx) -> int {
            while (sj + 1 < (int)nblocks && lds.spref[sj + 1] <= idx) sj++;
            return lds.sstart[sj] + (idx - lds.spref[sj]);
        };
        // a slice of one tile stays in registers for the item pass
        const bool one_tile = end - beg <= TILE;
        int u[SEL_U], pu[SEL_U], o0[SEL_U], o1[SEL_U];
#pragma unroll
        for (int k = 0; k < SEL_U; k++) u[k] = -1;  // an empty slice leaves no entries
        int s_run = 0, f_run = 0, i_run = 0;  // survivors, frontier and items so far (uniform)
        // the tile's entries; a tile's successor is loaded before the tile is
        // classified, so its round trip overlaps the classification
        // (round 0 visits every vertex: in id order, or under hub order in
        // spread_id order, which the alive lists then keep; the order by
        // round is then sorted after the loop)
        auto entry = [&](int idx) -> int {
            return (idx < end && map_ok) ? ((r == 0) ? (HUB ? spread_id(idx, a.n) : idx) : Lin[phys(idx)]) : -1;
        };
        // (and their priorities in the middle of the tile before)
        int un[SEL_U], pn[SEL_U];
#pragma unroll
        for (int k = 0; k < SEL_U; k++) un[k] = entry(beg + (int)threadIdx.x * SEL_U + k);
#pragma unroll
        for (int k = 0; k < SEL_U; k++) pn[k] = un[k] >= 0 ? a.prio[un[k]] : 0;
        for (int base = beg; base < end; base += TILE) {
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                u[k] = un[k];
                pu[k] = pn[k];
                un[k] = entry(base + TILE + (int)threadIdx.x * SEL_U + k);
            }
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                const bool fr = u[k] >= 0 && (long long)pu[k] <= thr;
                o0[k] = fr ? a.off[u[k]] : 0;
                o1[k] = fr ? a.off[u[k] + 1] : 0;
            }
#pragma unroll
            for (int k = 0; k < SEL_U; k++) pn[k] = un[k] >= 0 ? a.prio[un[k]] : 0;
            // packed per-thread counts: [survivors: bits 0-15][items: 16-31]
            unsigned int val = 0;
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                if (u[k] < 0) continue;
                if ((long long)pu[k] <= thr) {
                    a.rnd[u[k]] = r;
                    const int d = o1[k] - o0[k];
                    if (d > 0) {
                        val += 1u << 16;
                        my_edges += (unsigned long long)d;
                        atomicOr(&a.st2[u[k] >> 4], 2u << ((u[k] & 15) * 2));
                    }
                } else {
                    val += 1u;
                    lmin = min(lmin, (unsigned int)pu[k]);
                }
            }
            unsigned int tot;
            const unsigned int ex = block_excl_scan<PEEL_BLK>(val, &tot, shm);
            // every entry of the tile is a survivor or a frontier vertex (none
            // is read when the map failed its check)
            const int tile_n = map_ok ? min(TILE, end - base) : 0;
            const int before = min((int)threadIdx.x * SEL_U, tile_n);
            int sr = beg + s_run + (int)(ex & 0xFFFFu);
            int fr = end - 1 - (f_run + before - (int)(ex & 0xFFFFu));
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                if (u[k] < 0) continue;
                if ((long long)pu[k] > thr) {
                    Lout[sr++] = u[k];
                } else {
                    Lout[fr--] = u[k];
                }
            }
            s_run += (int)(tot & 0xFFFFu);
            f_run += tile_n - (int)(tot & 0xFFFFu);
            i_run += (int)(tot >> 16);
        }
        {
            const unsigned long long eb = block_sum<PEEL_BLK>(my_edges, shs);
            const unsigned long long packed = ((unsigned long long)i_run << FCNT_SHIFT) | eb;
            if (threadIdx.x == 0) {
                s_fbase = packed ? atomicAdd(&ctl->fcnt[slot], packed) : 0ull;
                if (s_run) atomicAdd(&ctl->lcnt[nslot], (unsigned int)s_run);
                seg_out[blockIdx.x] = beg;
                seg_out[PEEL_BLK + blockIdx.x] = s_run;
                seg_out[2 * PEEL_BLK + blockIdx.x] = f_run;
            }
            __syncthreads();  // also orders the tail writes before the reads below
        }
        unsigned long long fb = s_fbase;
        // item pass: the frontier vertices with edges, from registers (one
        // tile) or from the tail, placed at the reserved item range
        const int item_end = one_tile ? (end > beg ? 1 : 0) : f_run;  // one register pass, or the tail
        for (int base = 0; base < item_end; base += TILE) {
            if (!one_tile) {
#pragma unroll
                for (int k = 0; k < SEL_U; k++) {
                    const int j = base + (int)threadIdx.x * SEL_U + k;
                    u[k] = j < f_run ? Lout[end - 1 - j] : -1;
                }
#pragma unroll
                for (int k = 0; k < SEL_U; k++) {
                    o0[k] = u[k] >= 0 ? a.off[u[k]] : 0;
                    o1[k] = u[k] >= 0 ? a.off[u[k] + 1] : 0;
                    pu[k] = 0;  // every tail entry is a frontier vertex (those without edges are skipped)
                }
            }
            unsigned long long val = 0;
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                if (u[k] < 0 || (long long)pu[k] > thr) continue;
                const int d = o1[k] - o0[k];
                if (d > 0) val += (1ull << TITEM_SHIFT) + (unsigned long long)d;
            }
            unsigned long long tot;
            const unsigned long long ex = block_excl_scan<PEEL_BLK>(val, &tot, shs);
            unsigned long long it = (fb >> FCNT_SHIFT) + (ex >> TITEM_SHIFT);
            unsigned long long ed = (fb & FCNT_MASK) + (ex & 0xFFFFFFFFull);
#pragma unroll
            for (int k = 0; k < SEL_U; k++) {
                if (u[k] < 0 || (long long)pu[k] > thr) continue;
                const int d = o1[k] - o0[k];
                if (d > 0) {
                    ivr[it] = u[k];
                    a.ie[it] = (int)ed;
                    a.ir[it] = o0[k] - (int)ed;
                    mark_chunks<PEEL_MARK>((long long)ed, (long long)ed + d, (int)it, a.cfirst, a.clast);
                    it++;
                    ed += d;
                }
            }
            fb += ((tot >> TITEM_SHIFT) << FCNT_SHIFT) + (tot & 0xFFFFFFFFull);
        }
        grid_sync(bar);
        // ---------------- sweep
        const unsigned long long f = ld_agent_u64(&ctl->fcnt[slot]);
        const int K = (int)(f >> FCNT_SHIFT);
        const long long E = (long long)(f & FCNT_MASK);
        const bool bucket = a.nr > 0 && E >= a.bkt_min_e;
        PeelEdgeOp<PEEL_BLK> op{a.st2, a.prio, r, lmin, ctl, &lds.m.dec, bucket, a.bm, a.nr, a.n, a.rbase, a.bkt,
                                a.bfill, lds.bcnt, lds.bbase};
        op.hub = HUB;
        if (E >= a.coarse_min_e)
            sweep_chunks<PEEL_BLK, PEEL_CH, PEEL_CH / PEEL_MARK>(K, E, ivr, a.ie, a.ir, a.cfirst, a.clast, a.adj,
                                                                 a.inc, op, lds.m.sw, blockIdx.x, nblocks,
                                                                 &ctl->cnext[slot], &s_chunk);
        else
            sweep_chunks<PEEL_BLK, PEEL_MARK, 1>(K, E, ivr, a.ie, a.ir, a.cfirst, a.clast, a.adj, a.inc, op,
                                                 lds.m.sw, blockIdx.x, nblocks, &ctl->cnext[slot], &s_chunk);
        unsigned int rmin = op.lmin;
        if (bucket) {
            grid_sync(bar);
            // apply: block b owns ranges b, b + grid, ...  It sums each
            // range's bucket entries in a dense LDS histogram, then walks the
            // entries again: the first entry of each vertex takes (and
            // clears) its slot and lowers the priority with a plain
            // read-modify-write (no other block touches it until the next
            // grid sync).  Work follows the entries, not the range size, and
            // every range leaves the histogram clear for the next one.
            const DenseHist H{lds.dense, s_hubh, a.bm.hub >> a.bm.sb, HUB && a.narrow != 0, 1u << a.rshift};
            if ((int)blockIdx.x < a.nr) {
                H.clear(threadIdx.x, PEEL_BLK);  // it aliases the sweep's LDS
                lds_barrier();
            }
            for (int j = blockIdx.x; j < a.nr; j += nblocks) {
                const int lo = a.rbase[j];
                // a reservation past the range's capacity was refused (and
                // flagged) but still counted: never read past the range
                const int cnt = min((int)ld_agent(&a.bfill[j]), a.rbase[j + 1] - lo);
                for (int i = threadIdx.x; i < cnt; i += PEEL_BLK) {
                    const unsigned int e = (unsigned int)a.bkt[lo + i];
                    H.add(e >> BKT_CNT_BITS, (int)(e & ((1u << BKT_CNT_BITS) - 1)) + 1);
                }
                lds_barrier();
                for (int i = threadIdx.x; i < cnt; i += PEEL_BLK) {
                    const unsigned int li = (unsigned int)a.bkt[lo + i] >> BKT_CNT_BITS;
                    if (li < H.limit) {
                        const int c = H.take(li);
                        const int u = a.bm.global(j, (int)li);
                        if (c && u < a.n) {
                            const int pu = a.prio[u] - c;
                            a.prio[u] = pu;
                            rmin = min(rmin, (unsigned int)pu);
                        }
                    }
                }
                if (threadIdx.x == 0) a.bfill[j] = 0;  // empty for the next bucketed round
                lds_barrier();
            }
            if ((int)blockIdx.x < a.nr) {
                // the histogram overwrote the decrement table
                for (int t = threadIdx.x; t < DEC_SLOTS; t += PEEL_BLK) {
                    lds.m.dec.key[t] = DEC_EMPTY;
                    lds.m.dec.cnt[t] = 0;
                }
            }
        }
        const unsigned int bmin = block_min<PEEL_BLK>(rmin, shm);
        if (threadIdx.x == 0 && bmin != 0xFFFFFFFFu) atomicMin(&ctl->mn[nslot], bmin);
        {
            // This round's segment table was published by the grid sync after
            // the select, so the next round's mapping is built while the
            // round-end barrier completes: the loads share the barrier's wait
            // for outstanding memory operations, the scan runs between its
            // halves.  The same scan gives this block's place in the round's
            // frontier: positions follow rounds, and ascending id inside a
            // round, which is block order and then slice order; the vertices
            // peeled before this round hold the first n - Lc positions.
            const int* __restrict__ seg_next = a.seg + (r & 1) * 3 * PEEL_BLK;
            const int j = (int)threadIdx.x;
            const int len = j < (int)nblocks ? seg_next[PEEL_BLK + j] : 0;
            const int st = j < (int)nblocks ? seg_next[j] : 0;
            const int fl = j < (int)nblocks ? seg_next[2 * PEEL_BLK + j] : 0;
            grid_arrive(bar);
            unsigned long long tot;
            // [alive entries: bits 0-31][frontier: 32-63]; each sum is below 2^31
            const unsigned long long ex = block_excl_scan<PEEL_BLK>(
                ((unsigned long long)(unsigned int)fl << 32) | (unsigned int)len, &tot, shs);
            if (j < (int)nblocks) {
                lds.spref[j] = (int)(ex & 0xFFFFFFFFull);
                lds.sstart[j] = st;
            }
            if (j == 0) s_segtot = tot & 0xFFFFFFFFull;
            if (j == (int)blockIdx.x) s_fbase = (unsigned long long)(a.n - Lc) + (ex >> 32);
            __syncthreads();
            const long long fb0 = (long long)s_fbase;
            for (int i = j; i < f_run; i += PEEL_BLK) {
                const long long p = fb0 + i;
                if (p < a.n) {
                    a.order[p] = Lout[end - 1 - i];
                } else if (i == j) {
                    atomicAdd(&ctl->err_count, 1);
                    ctl->err_code = ERR_INTERNAL;
                }
            }
            grid_wait(bar);
        }
    }
}

// ============================================================ near-list PEEL
// The same round loop with a select that does not rescan every alive vertex in
// every round.  Large sparse graphs have hundreds of rounds per iteration in
// which millions of vertices are alive and a few hundred are peeled; the
// full-list select reads every alive vertex in each of them.  Here:
//   * the near bound B splits the alive vertices.  The near list N holds
//     exactly the alive vertices whose priority is at most B.  Priorities
//     only fall within an iteration, so a vertex joins N at most once: when a
//     decrement first takes its priority from above B to B or below, the
//     decrement appends it to the crossing list X, which the next round reads
//     after N's own entries;
//   * a round whose threshold is at most B has its whole frontier in N and
//     scans only N.  Every other round (round 0, a threshold above B, or an
//     empty N) scans the full list F, sets B = thr * near_num / near_den +
//     near_add and rebuilds N.  F is compacted (the vertices peeled since it
//     was last written dropped) only once more than a quarter of it is
//     peeled, and is not stored at all before its first compaction;
//   * the next round's minimum is exact whenever N is not empty: every near
//     vertex bids its priority, and every other alive vertex is above B.  When
//     N runs empty, the next round first rescans F for the exact minimum (one
//     more pass over F and one more grid sync), then classifies F;
//   * under hub order the first pass visits the ids in spread_id order, which
//     F keeps, so that every block's slice samples the whole id space;
//   * peeled vertices get priority -1, which marks them dead in F;
//   * a round's frontier comes out of N in list order, not id order, so the
//     positions (by round, ascending id inside a round) are sorted after the
//     loop instead of written by it.
// Rounds, frontiers, charges and decrements are those of k_peel_rounds.
// Lists are virtual as there: each block writes its outputs to its own
// segment (at its slice's start), and per-block tables of segment starts and
// lengths map virtual positions.

// 512 threads per block: at 1024 the kernel spilled about 45 VGPRs and its
// sweep paid for it (53.1 ms per iteration on the 40M-vertex Chung-Lu graph);
// at 512 it spills none (48.9 ms).  Four list entries per thread per tile.
constexpr int NEAR_BLK = 512;
constexpr int NEAR_SEL_U = 4;
constexpr int SEG_STRIDE = PEEL_BLK;  // segment tables hold PEEL_BLK entries per field
constexpr int APPLY_META = 64;        // ranges per block whose bounds are read up front (2048 ranges / 32 blocks)
constexpr int APPLY_REG = 8;          // bucket entries per thread kept in registers between the apply's passes
constexpr int NEAR_PF = 2;            // items per thread of the next sweep chunk loaded ahead
using PeelSweepLdsT = SweepLds<PEEL_CH>;
static_assert(NEAR_BLK * NEAR_SEL_U < (1 << 16), "tile counts must fit their packed fields");
static_assert(DEC_SLOTS % NEAR_BLK == 0, "slots must be a multiple of the block");

// LDS map of a segment table tab[start | len][SEG_STRIDE] with nseg segments;
// returns the total length.  Reads of `tab` must follow the grid barrier
// that published it.  Contains block barriers.
__device__ __forceinline__ long long build_map(const int* __restrict__ tab, int nseg, int* spref, int* sstart,
                                               unsigned long long* shs) {
    const int j = (int)threadIdx.x;
    const int len = j < nseg ? tab[SEG_STRIDE + j] : 0;
    const int st = j < nseg ? tab[j] : 0;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<NEAR_BLK>((unsigned long long)(unsigned int)len, &tot, shs);
    if (j < nseg) {
        spref[j] = (int)ex;
        sstart[j] = st;
    }
    __syncthreads();
    return (long long)tot;
}

// Per-block result of one classification pass over a list slice.
struct NearPass {
    int n_run;   // near survivors written to the near segment
    int s_run;   // survivors written to the full-list segment
    int f_run;   // frontier vertices (written to the tail of the near slice)
    int i_run;   // frontier vertices with edges
    unsigned long long edges;  // frontier edges (this thread's share)
    unsigned int lmin;         // smallest survivor priority (this thread's share)
    bool one_tile;
};

// Classifies the slice [beg, end) of a virtual list.  kind 0: entry i is
// vertex i (spread_id(i) under hub order); 1: Lin[map(i)]; 2: Lin[map(i)] for
// i < mtot, then Xin[i - mtot].
// Each alive entry (priority >= 0) goes to exactly one class:
//   frontier (priority <= thr): round r, priority -1, state bit, Nout tail;
//   survivor: bids its priority; to Fout[beg + ...] when Fout is given, and
//   to Nout[beg + ...] when its priority is at most B.
// For slices of one tile the frontier stays in registers (u, fr, o0, o1).
template <bool WRITE_F>
__device__ __forceinline__ NearPass near_classify(const PeelArgs& a, int r, int kind, const int* __restrict__ Lin,
                                                  const int* __restrict__ Xin, long long mtot, int beg, int end,
                                                  long long thr, long long B, int* __restrict__ Fout,
                                                  int* __restrict__ Nout, const int* spref, const int* sstart,
                                                  unsigned long long* shs, int (&u)[NEAR_SEL_U], bool (&fr)[NEAR_SEL_U],
                                                  int (&o0)[NEAR_SEL_U], int (&o1)[NEAR_SEL_U]) {
    constexpr int TILE = NEAR_BLK * NEAR_SEL_U;
    const int nseg = (int)gridDim.x;
    NearPass P{0, 0, 0, 0, 0ull, 0xFFFFFFFFu, end - beg <= TILE};
    int sj = 0;
    if (kind != 0 && end > beg) {
        const int first = beg + (int)threadIdx.x * NEAR_SEL_U;
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (spref[mid] <= first) lo = mid; else hi = mid - 1;
        }
        sj = lo;
    }
    auto entry = [&](int idx) -> int {
        if (idx >= end) return -1;
        if (kind == 0) return a.hub ? spread_id(idx, a.n) : idx;
        if (kind == 2 && idx >= mtot) return Xin[idx - mtot];
        while (sj + 1 < nseg && spref[sj + 1] <= idx) sj++;
        return Lin[sstart[sj] + (idx - spref[sj])];
    };
    // The next tile's entries are loaded at the top of a tile and their
    // priorities in its middle, so a tile waits on neither.  (No block writes
    // the priority of a vertex in another slice during the select.)
    int un[NEAR_SEL_U], pn[NEAR_SEL_U];
#pragma unroll
    for (int k = 0; k < NEAR_SEL_U; k++) {
        u[k] = -1;
        fr[k] = false;
        un[k] = entry(beg + (int)threadIdx.x * NEAR_SEL_U + k);
    }
#pragma unroll
    for (int k = 0; k < NEAR_SEL_U; k++) pn[k] = un[k] >= 0 ? a.prio[un[k]] : -1;
    for (int base = beg; base < end; base += TILE) {
        int pu[NEAR_SEL_U];
#pragma unroll
        for (int k = 0; k < NEAR_SEL_U; k++) {
            u[k] = un[k];
            pu[k] = pn[k];
            un[k] = entry(base + TILE + (int)threadIdx.x * NEAR_SEL_U + k);
        }
#pragma unroll
        for (int k = 0; k < NEAR_SEL_U; k++) {
            fr[k] = pu[k] >= 0 && (long long)pu[k] <= thr;
            o0[k] = fr[k] ? a.off[u[k]] : 0;
            o1[k] = fr[k] ? a.off[u[k] + 1] : 0;
        }
#pragma unroll
        for (int k = 0; k < NEAR_SEL_U; k++) pn[k] = un[k] >= 0 ? a.prio[un[k]] : -1;
        // packed per-thread counts: [near: 0-15][full-list survivors: 16-31][frontier: 32-47][items: 48-63]
        unsigned long long val = 0;
        // frontier marks of this thread's entries, one atomic per state word
        int mword = -1;
        unsigned int mbits = 0;
#pragma unroll
        for (int k = 0; k < NEAR_SEL_U; k++) {
            if (pu[k] < 0) continue;  // no entry, or peeled in an earlier round
            if (fr[k]) {
                a.rnd[u[k]] = r;
                a.prio[u[k]] = -1;
                val += 1ull << 32;
                const int d = o1[k] - o0[k];
                if (d > 0) {
                    val += 1ull << 48;
                    P.edges += (unsigned long long)d;
                    if ((u[k] >> 4) != mword) {
                        if (mbits) atomicOr(&a.st2[mword], mbits);
                        mword = u[k] >> 4;
                        mbits = 0;
                    }
                    mbits |= 2u << ((u[k] & 15) * 2);
                }
            } else {
                P.lmin = min(P.lmin, (unsigned int)pu[k]);
                if (WRITE_F) val += 1ull << 16;
                if ((long long)pu[k] <= B) val += 1ull;
            }
        }
        if (mbits) atomicOr(&a.st2[mword], mbits);
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan<NEAR_BLK>(val, &tot, shs);
        int nr_ = beg + P.n_run + (int)(ex & 0xFFFFull);
        int sr_ = beg + P.s_run + (int)((ex >> 16) & 0xFFFFull);
        int fr_ = end - 1 - (P.f_run + (int)((ex >> 32) & 0xFFFFull));
#pragma unroll
        for (int k = 0; k < NEAR_SEL_U; k++) {
            if (pu[k] < 0) continue;
            if (fr[k]) {
                Nout[fr_--] = u[k];
            } else {
                if (WRITE_F) Fout[sr_++] = u[k];
                if ((long long)pu[k] <= B) Nout[nr_++] = u[k];
            }
        }
        P.n_run += (int)(tot & 0xFFFFull);
        P.s_run += (int)((tot >> 16) & 0xFFFFull);
        P.f_run += (int)((tot >> 32) & 0xFFFFull);
        P.i_run += (int)(tot >> 48);
    }
    return P;
}

template <bool MONO>
__global__ __launch_bounds__(NEAR_BLK, 1) void k_peel_rounds_near(PeelArgs a) {
    __shared__ PeelLds lds;
    __shared__ unsigned long long shs[NEAR_BLK / WAVE];
    __shared__ unsigned int shm[NEAR_BLK / WAVE];
    __shared__ unsigned long long s_fbase;
    __shared__ int s_chunk;
    __shared__ long long s_ntot;  // entries in the near list's segments (map built at the previous round's end)
    __shared__ unsigned int s_xn;     // staged crossings
    __shared__ int s_meta[2 * APPLY_META];  // bucket apply: start and entry count of each of the block's ranges
    __shared__ int s_hubh[BKT_HUB_IDS >> BKT_NARROW_MIN_SB];  // narrow apply: the hubs' counters
    __shared__ unsigned int s_xbase;  // their reserved start in the global list
    Ctl* ctl = a.ctl;
    GridSync* gs = a.gs;
    const unsigned int nblocks = gridDim.x;
    const long long q = a.eps_den, p = a.eps_num;
    for (int slot = threadIdx.x; slot < DEC_SLOTS; slot += NEAR_BLK) {
        lds.m.dec.key[slot] = DEC_EMPTY;
        lds.m.dec.cnt[slot] = 0;
    }
    for (int j = threadIdx.x; j < BKT_MAX_NR; j += NEAR_BLK) lds.bcnt[j] = 0;
    if (threadIdx.x == 0) {
        s_ntot = 0;
        s_xn = 0;
    }
    GridBarrier bar = grid_sync_init(gs, nblocks, xcd_id());
    long long alive = a.n;
    long long B = -1;        // near bound (-1 until the first full-list round)
    long long thr_prev = 0;  // MONO: largest threshold so far
    int fpar = 0;            // the full list F is segF[fpar] over L0 (fpar 0) or L1 (fpar 1)
    bool f_all = true;       // F is still every vertex (before the first full-list round writes it)
    for (int r = 0;; r++) {
        const int slot = r & 3, nslot = (r + 1) & 3;
        if (r > 0) {
            const unsigned int pc = ld_agent(&ctl->pcnt[(r - 1) & 3]);
            if (pc == 0u || (long long)pc > alive) {
                // every round peels the minimum vertex; all blocks see the same
                // counts and leave together
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    ctl->nrounds = r;
                    atomicAdd(&ctl->err_count, 1);
                    ctl->err_code = ERR_INTERNAL;
                }
                break;
            }
            alive -= pc;
        }
        if (alive == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) ctl->nrounds = r;
            break;
        }
        unsigned int mn = ld_agent(&ctl->mn[slot]);
        const long long xin = r > 0 ? (long long)ld_agent(&ctl->xcnt[slot]) : 0;
        const long long nin = r > 0 ? s_ntot + xin : 0;
        long long thr = ((q + p) * (long long)mn) / q;
        if (MONO && r > 0) thr = max(thr, thr_prev);
        const bool full = r == 0 || nin == 0 || thr > B;
        const bool exact = r == 0 || nin > 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int zs = (r + 2) & 3;
            ctl->mn[zs] = 0xFFFFFFFFu;
            ctl->fcnt[zs] = 0;
            ctl->cnext[zs] = 0;
            ctl->pcnt[zs] = 0;
            ctl->xcnt[zs] = 0;
            ctl->mn2[zs] = 0xFFFFFFFFu;
        }
        int* __restrict__ ivr = (r & 1) ? a.iv1 : a.iv0;
        const int* __restrict__ Nin = (r & 1) ? a.N1 : a.N0;
        int* __restrict__ Nout = (r & 1) ? a.N0 : a.N1;
        const int* __restrict__ Xin = (r & 1) ? a.X1 : a.X0;
        int* __restrict__ Xout = (r & 1) ? a.X0 : a.X1;
        int* __restrict__ segNout = a.segN + (r & 1) * 2 * SEG_STRIDE;
        if (r > 0) {
            // the previous round's frontier is peeled now: clear its state bits
            const int* __restrict__ ivp = (r & 1) ? a.iv0 : a.iv1;
            const int Kp = (int)(ld_agent_u64(&ctl->fcnt[(r - 1) & 3]) >> FCNT_SHIFT);
            for (int k = blockIdx.x * NEAR_BLK + threadIdx.x; k < Kp; k += nblocks * NEAR_BLK) {
                const int w = ivp[k];
                atomicAnd(&a.st2[w >> 4], ~(3u << ((w & 15) * 2)));
            }
        }
        int u[NEAR_SEL_U], o0[NEAR_SEL_U], o1[NEAR_SEL_U];
        bool fr[NEAR_SEL_U];
        NearPass P;
        int beg, end;
        if (full) {
            long long ftot = a.n;
            if (!f_all) ftot = build_map(a.segF + fpar * 2 * SEG_STRIDE, (int)nblocks, lds.spref, lds.sstart, shs);
            // F is compacted (its survivors written to the other buffer) only
            // once more than a quarter of its entries are peeled; until then a
            // full-list pass reads it as it is (a peeled vertex has priority
            // -1), and before the first compaction it reads no list at all
            const bool compact = ftot - alive > ftot / 4;
            if (!exact) {
                // N ran empty: find the exact minimum first
                const long long per = (ftot + nblocks - 1) / nblocks;
                beg = (int)min(ftot, (long long)blockIdx.x * per);
                end = (int)min(ftot, (long long)beg + per);
                const int* Fin = fpar ? a.L1 : a.L0;
                if (compact) {
                    int* Fout = fpar ? a.L0 : a.L1;
                    P = near_classify<true>(a, r, f_all ? 0 : 1, Fin, nullptr, ftot, beg, end, -2, -1, Fout, Nout,
                                            lds.spref, lds.sstart, shs, u, fr, o0, o1);
                    int* segFout = a.segF + (fpar ^ 1) * 2 * SEG_STRIDE;
                    if (threadIdx.x == 0) {
                        segFout[blockIdx.x] = beg;
                        segFout[SEG_STRIDE + blockIdx.x] = P.s_run;
                    }
                } else {
                    P = near_classify<false>(a, r, f_all ? 0 : 1, Fin, nullptr, ftot, beg, end, -2, -1, nullptr, Nout,
                                             lds.spref, lds.sstart, shs, u, fr, o0, o1);
                }
                const unsigned int bmin = block_min<NEAR_BLK>(P.lmin, shm);
                if (threadIdx.x == 0 && bmin != 0xFFFFFFFFu) atomicMin(&ctl->mn2[slot], bmin);
                grid_sync(bar);
                if (compact) {
                    fpar ^= 1;
                    f_all = false;
                    ftot = build_map(a.segF + fpar * 2 * SEG_STRIDE, (int)nblocks, lds.spref, lds.sstart, shs);
                }
                mn = ld_agent(&ctl->mn2[slot]);
                thr = ((q + p) * (long long)mn) / q;
                if (MONO && r > 0) thr = max(thr, thr_prev);
            }
            B = min(thr * a.near_num / a.near_den + a.near_add, (long long)0x7FFFFFFE);
            const long long per = (ftot + nblocks - 1) / nblocks;
            beg = (int)min(ftot, (long long)blockIdx.x * per);
            end = (int)min(ftot, (long long)beg + per);
            const int* Fin = fpar ? a.L1 : a.L0;
            if (exact && compact) {
                // one pass: survivors to the other F buffer, near survivors to N
                int* Fout = fpar ? a.L0 : a.L1;
                P = near_classify<true>(a, r, f_all ? 0 : 1, Fin, nullptr, ftot, beg, end, thr, B, Fout, Nout,
                                        lds.spref, lds.sstart, shs, u, fr, o0, o1);
                int* segFout = a.segF + (fpar ^ 1) * 2 * SEG_STRIDE;
                if (threadIdx.x == 0) {
                    segFout[blockIdx.x] = beg;
                    segFout[SEG_STRIDE + blockIdx.x] = P.s_run;
                }
                fpar ^= 1;
                f_all = false;
            } else {
                P = near_classify<false>(a, r, f_all ? 0 : 1, Fin, nullptr, ftot, beg, end, thr, B, nullptr, Nout,
                                         lds.spref, lds.sstart, shs, u, fr, o0, o1);
            }
        } else {
            const long long per = (nin + nblocks - 1) / nblocks;
            beg = (int)min(nin, (long long)blockIdx.x * per);
            end = (int)min(nin, (long long)beg + per);
            P = near_classify<false>(a, r, 2, Nin, Xin, s_ntot, beg, end, thr, B, nullptr, Nout, lds.spref,
                                     lds.sstart, shs, u, fr, o0, o1);
        }
        thr_prev = thr;
        if (a.rmin && blockIdx.x == 0 && threadIdx.x == 0) a.rmin[r] = (int)min(thr, 0x7FFFFFFFLL);
        {
            const unsigned long long eb = block_sum<NEAR_BLK>(P.edges, shs);
            const unsigned long long packed = ((unsigned long long)P.i_run << FCNT_SHIFT) | eb;
            if (threadIdx.x == 0) {
                s_fbase = packed ? atomicAdd(&ctl->fcnt[slot], packed) : 0ull;
                if (P.f_run) atomicAdd(&ctl->pcnt[slot], (unsigned int)P.f_run);
                segNout[blockIdx.x] = beg;
                segNout[SEG_STRIDE + blockIdx.x] = P.n_run;
            }
            __syncthreads();  // also orders the tail writes before the reads below
        }
        unsigned long long fb = s_fbase;
        // item pass: the frontier vertices with edges, from registers (one
        // tile) or from the tail of the block's near slice
        constexpr int TILE = NEAR_BLK * NEAR_SEL_U;
        const int item_end = P.one_tile ? (end > beg ? 1 : 0) : P.f_run;
        for (int base = 0; base < item_end; base += TILE) {
            if (!P.one_tile) {
#pragma unroll
                for (int k = 0; k < NEAR_SEL_U; k++) {
                    const int j = base + (int)threadIdx.x * NEAR_SEL_U + k;
                    u[k] = j < P.f_run ? Nout[end - 1 - j] : -1;
                    fr[k] = u[k] >= 0;
                    o0[k] = fr[k] ? a.off[u[k]] : 0;
                    o1[k] = fr[k] ? a.off[u[k] + 1] : 0;
                }
            }
            unsigned long long val = 0;
#pragma unroll
            for (int k = 0; k < NEAR_SEL_U; k++) {
                const int d = o1[k] - o0[k];
                if (fr[k] && d > 0) val += (1ull << TITEM_SHIFT) + (unsigned long long)d;
            }
            unsigned long long tot;
            const unsigned long long ex = block_excl_scan<NEAR_BLK>(val, &tot, shs);
            unsigned long long it = (fb >> FCNT_SHIFT) + (ex >> TITEM_SHIFT);
            unsigned long long ed = (fb & FCNT_MASK) + (ex & 0xFFFFFFFFull);
#pragma unroll
            for (int k = 0; k < NEAR_SEL_U; k++) {
                const int d = o1[k] - o0[k];
                if (fr[k] && d > 0) {
                    ivr[it] = u[k];
                    a.ie[it] = (int)ed;
                    a.ir[it] = o0[k] - (int)ed;
                    mark_chunks<PEEL_MARK>((long long)ed, (long long)ed + d, (int)it, a.cfirst, a.clast);
                    it++;
                    ed += d;
                }
            }
            fb += ((tot >> TITEM_SHIFT) << FCNT_SHIFT) + (tot & 0xFFFFFFFFull);
        }
        grid_sync(bar);
        // ---------------- sweep
        const unsigned long long f = ld_agent_u64(&ctl->fcnt[slot]);
        const int K = (int)(f >> FCNT_SHIFT);
        const long long E = (long long)(f & FCNT_MASK);
        const bool bucket = a.nr > 0 && E >= a.bkt_min_e;
        PeelEdgeOp<NEAR_BLK> op{a.st2, a.prio, r, P.lmin, ctl, &lds.m.dec, bucket, a.bm, a.nr, a.n, a.rbase, a.bkt, a.bfill,
                      lds.bcnt, lds.bbase};
        // crossings are staged in lds.bbase, which only the bucket flush uses (as scratch)
        const XStage xst{lds.bbase, &s_xn, Xout, &ctl->xcnt[nslot], a.n, ctl};
        op.nearB = (int)B;
        op.xst = xst;
        op.hub = a.hub != 0;
        if (E >= a.coarse_min_e)
            sweep_chunks<NEAR_BLK, PEEL_CH, PEEL_CH / PEEL_MARK, PeelEdgeOp<NEAR_BLK>, PeelSweepLdsT, NEAR_PF>(
                K, E, ivr, a.ie, a.ir, a.cfirst, a.clast, a.adj,
                                                                 a.inc, op, lds.m.sw, blockIdx.x, nblocks,
                                                                 &ctl->cnext[slot], &s_chunk);
        else
            sweep_chunks<NEAR_BLK, PEEL_MARK, 1, PeelEdgeOp<NEAR_BLK>, PeelSweepLdsT, NEAR_PF>(
                K, E, ivr, a.ie, a.ir, a.cfirst, a.clast, a.adj, a.inc, op,
                                                 lds.m.sw, blockIdx.x, nblocks, &ctl->cnext[slot], &s_chunk);
        unsigned int rmin = op.lmin;
        if (bucket) {
            grid_sync(bar);
            // apply the owner buckets as k_peel_rounds does, with two memory
            // round trips fewer per range: the block reads the bounds and fill
            // counts of all its ranges at once, and keeps up to
            // APPLY_REG * NEAR_BLK entries of a range in registers between the
            // two passes.  A decrement that crosses B appends its vertex to the
            // crossing list.
            const DenseHist H{lds.dense, s_hubh, a.bm.hub >> a.bm.sb, a.narrow != 0, 1u << a.rshift};
            const int my_nr = (int)blockIdx.x < a.nr ? (a.nr - (int)blockIdx.x + (int)nblocks - 1) / (int)nblocks : 0;
            if (my_nr > 0) {
                for (int t = threadIdx.x; t < min(my_nr, APPLY_META); t += NEAR_BLK) {
                    const int j = (int)blockIdx.x + t * (int)nblocks;
                    const int lo = a.rbase[j];
                    s_meta[2 * t] = lo;
                    // a reservation past the range's capacity was refused (and
                    // flagged) but still counted: never read past the range
                    s_meta[2 * t + 1] = min((int)ld_agent(&a.bfill[j]), a.rbase[j + 1] - lo);
                }
                H.clear(threadIdx.x, NEAR_BLK);  // it aliases the sweep's LDS
                lds_barrier();
            }
            for (int k = 0; k < my_nr; k++) {
                const int j = (int)blockIdx.x + k * (int)nblocks;
                int lo, cnt;
                if (k < APPLY_META) {
                    lo = s_meta[2 * k];
                    cnt = s_meta[2 * k + 1];
                } else {
                    lo = a.rbase[j];
                    cnt = min((int)ld_agent(&a.bfill[j]), a.rbase[j + 1] - lo);
                }
                constexpr unsigned int CMASK = (1u << BKT_CNT_BITS) - 1;
                unsigned int ent[APPLY_REG];
#pragma unroll
                for (int q = 0; q < APPLY_REG; q++) {
                    const int i = (int)threadIdx.x + q * NEAR_BLK;
                    ent[q] = i < cnt ? (unsigned int)a.bkt[lo + i] : 0xFFFFFFFFu;  // local id 2^20 - 1: no slot
                }
#pragma unroll
                for (int q = 0; q < APPLY_REG; q++) H.add(ent[q] >> BKT_CNT_BITS, (int)(ent[q] & CMASK) + 1);
                for (int i = (int)threadIdx.x + APPLY_REG * NEAR_BLK; i < cnt; i += NEAR_BLK) {
                    const unsigned int e = (unsigned int)a.bkt[lo + i];
                    H.add(e >> BKT_CNT_BITS, (int)(e & CMASK) + 1);
                }
                lds_barrier();
                // the first entry of each vertex takes (and clears) its slot
                auto take = [&](unsigned int e) {
                    bool x = false;
                    int w = 0;
                    const unsigned int li = e >> BKT_CNT_BITS;
                    if (li < H.limit) {
                        const int c = H.take(li);
                        const int u = a.bm.global(j, (int)li);
                        if (c && u < a.n) {
                            w = u;
                            const int old = a.prio[w];
                            const int pw = old - c;
                            a.prio[w] = pw;
                            rmin = min(rmin, (unsigned int)pw);
                            x = (long long)old > B && (long long)pw <= B;
                        }
                    }
                    xst.stage_wave(x, w);
                };
#pragma unroll
                for (int q = 0; q < APPLY_REG; q++) take(ent[q]);
                for (int base = APPLY_REG * NEAR_BLK; base < cnt; base += NEAR_BLK) {
                    const int i = base + (int)threadIdx.x;
                    take(i < cnt ? (unsigned int)a.bkt[lo + i] : 0xFFFFFFFFu);
                }
                lds_barrier();
            }
            for (int t = threadIdx.x; t < my_nr; t += NEAR_BLK) a.bfill[(int)blockIdx.x + t * (int)nblocks] = 0;
            if ((int)blockIdx.x < a.nr) {
                for (int t = threadIdx.x; t < DEC_SLOTS; t += NEAR_BLK) {
                    lds.m.dec.key[t] = DEC_EMPTY;
                    lds.m.dec.cnt[t] = 0;
                }
            }
        }
        xst.flush(&s_xbase);
        const unsigned int bmin = block_min<NEAR_BLK>(rmin, shm);
        if (threadIdx.x == 0 && bmin != 0xFFFFFFFFu) atomicMin(&ctl->mn[nslot], bmin);
        {
            // the near list's segment table was published by the grid sync
            // after the select: map it between the halves of the round-end
            // barrier (the crossings' count is read after it)
            const int j = (int)threadIdx.x;
            const int len = j < (int)nblocks ? segNout[SEG_STRIDE + j] : 0;
            const int st = j < (int)nblocks ? segNout[j] : 0;
            grid_arrive(bar);
            unsigned long long tot;
            const unsigned long long ex =
                block_excl_scan<NEAR_BLK>((unsigned long long)(unsigned int)len, &tot, shs);
            if (j < (int)nblocks) {
                lds.spref[j] = (int)ex;
                lds.sstart[j] = st;
            }
            if (j == 0) s_ntot = (long long)tot;
            grid_wait(bar);
        }
    }
}

// ============================================================== SORT
// Coarse ranks: 16 position classes of about equal degree mass, as 4-bit
// codes packed 8 to a word and indexed by vertex (n/2 bytes, so a 4M-vertex
// table stays in each XCD's L2).  The class is non-decreasing in the
// position, so different classes order two vertices; only equal classes
// need the full positions.  The class bounds come from every 2^k-th
// position of the order (the smallest k leaving at most 2^17 samples): the
// degree mass of the sampled vertices is prefix-summed and class c starts at
// the first sample whose running mass reaches c/16 of the total (a sampling
// error only costs more ties).
constexpr int CR_MAX_SAMPLES = 1 << 17;
constexpr int CR_CLASSES = 16;
__host__ __device__ inline int cr_shift(int n) {
    int k = 0;
    while (((long long)n + (1LL << k) - 1) >> k > CR_MAX_SAMPLES) k++;
    return k;
}
constexpr int CR_POS_BITS = 28;  // staged word: class << 28 | position (n < 2^26)

// pos[order[i]] = i (kept in rnd[], which is the "round" of SORT), charge 0;
// with `sdeg`, also the degree of the vertex at each sampled position.
__global__ void k_sort_pos(int n, const int* __restrict__ order, int* __restrict__ rnd, int* __restrict__ inc,
                           const int* __restrict__ off, int* __restrict__ sdeg, int sshift) {
    const int smask = (1 << sshift) - 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = order[i];
        rnd[v] = i;
        inc[i] = 0;
        if (sdeg && (i & smask) == 0) sdeg[i >> sshift] = off[v + 1] - off[v];
    }
}

// Class bounds in two launches: k_coarse_tiles sums the sampled degree
// mass per tile of 1024 samples (one block per tile, coalesced), then
// k_coarse_bounds (one block) scans the tile sums and, for each class c,
// one wave scans the tile holding threshold c/16 of the total mass to find
// the crossing sample.
constexpr int CR_TILE = 1024;
constexpr int CR_MAX_TILES = CR_MAX_SAMPLES / CR_TILE;
static_assert(CR_MAX_TILES <= 1024 && (CR_CLASSES - 1) * WAVE <= 1024, "one block scans the tiles, a wave per class");

__global__ __launch_bounds__(CR_TILE) void k_coarse_tiles(int n, int sshift, const int* __restrict__ sdeg,
                                                          long long* __restrict__ tsum) {
    __shared__ long long sh[CR_TILE / WAVE];
    const int S = (int)(((long long)n + (1LL << sshift) - 1) >> sshift);
    const int i = (int)blockIdx.x * CR_TILE + (int)threadIdx.x;
    const long long t = block_sum<CR_TILE>((long long)(i < S ? sdeg[i] : 0), sh);
    if (threadIdx.x == 0) tsum[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_coarse_bounds(int n, int sshift, const int* __restrict__ sdeg,
                                                        const long long* __restrict__ tsum, int* __restrict__ bounds) {
    __shared__ long long sh[1024 / WAVE];
    __shared__ long long s_tex[CR_MAX_TILES];
    __shared__ long long s_tsum[CR_MAX_TILES];
    const int S = (int)(((long long)n + (1LL << sshift) - 1) >> sshift);
    const int nt = (S + CR_TILE - 1) / CR_TILE;
    const long long v = (int)threadIdx.x < nt ? tsum[threadIdx.x] : 0;
    long long tot;
    const long long ex = block_excl_scan<1024>(v, &tot, sh);
    if ((int)threadIdx.x < nt) {
        s_tex[threadIdx.x] = ex;
        s_tsum[threadIdx.x] = v;
    }
    __syncthreads();
    // class c starts at the first sample whose running mass reaches
    // floor(tot * c / 16); a zero threshold (or no mass) leaves the class empty
    const int c = (int)threadIdx.x / WAVE + 1;
    const int lane = (int)threadIdx.x & (WAVE - 1);
    if (threadIdx.x == 0) bounds[0] = 0;
    if (c >= CR_CLASSES) return;
    const long long th = (tot * c) / CR_CLASSES;
    int bound = n;
    if (th > 0) {
        // the tile whose mass interval (ex, ex + sum] holds th: exactly one
        int tile = -1;
        for (int t = lane; t < nt; t += WAVE)
            if (s_tex[t] < th && th <= s_tex[t] + s_tsum[t]) tile = t;
        for (int o = WAVE / 2; o > 0; o >>= 1) tile = max(tile, __shfl_xor(tile, o, WAVE));
        // lane l scans samples [l*16, l*16 + 16) of the tile
        constexpr int PL = CR_TILE / WAVE;
        const int s0 = tile * CR_TILE + lane * PL;
        int d[PL];
        long long mine = 0;
#pragma unroll
        for (int k = 0; k < PL; k++) {
            d[k] = s0 + k < S ? sdeg[s0 + k] : 0;
            mine += d[k];
        }
        long long run = s_tex[tile] + wave_incl_scan(mine) - mine;
        int hit = -1;
#pragma unroll
        for (int k = 0; k < PL; k++) {
            if (run < th && th <= run + d[k]) hit = s0 + k;
            run += d[k];
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) hit = max(hit, __shfl_xor(hit, o, WAVE));
        if (hit >= 0) bound = hit << sshift;
    }
    if (lane == 0) bounds[c] = bound;
}

__global__ void k_coarse_pack(int n, const int* __restrict__ pos, const int* __restrict__ bounds,
                              unsigned int* __restrict__ cb) {
    int b[CR_CLASSES];
#pragma unroll
    for (int c = 0; c < CR_CLASSES; c++) b[c] = bounds[c];
    const int words = (n + 7) / 8;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
        unsigned int word = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int v = w * 8 + k;
            if (v < n) {
                const int p = pos[v];
                unsigned int cls = 0;
#pragma unroll
                for (int c = 1; c < CR_CLASSES; c++) cls += p >= b[c] ? 1u : 0u;
                word |= cls << (4 * k);
            }
        }
        cb[w] = word;
    }
}

struct SortEdgeOp {
    const int* pos;
    const unsigned int* cb;  // coarse ranks, or null (compare positions directly)
    Ctl* ctl;
    int* spos;  // LDS: per staged item, its position (and class << 28 with coarse ranks)
    __device__ void flag_error() {
        atomicAdd(&ctl->err_count, 1);
        ctl->err_code = ERR_INTERNAL;
    }
    __device__ __forceinline__ int cls(int u) const { return (int)((cb[u >> 3] >> ((u & 7) * 4)) & 15u); }
    __device__ __forceinline__ void stage_item(int j, int v) {
        spos[j] = cb ? (int)(((unsigned int)cls(v) << CR_POS_BITS) | (unsigned int)pos[v]) : pos[v];
    }
    __device__ __forceinline__ int gather(int u) const { return cb ? cls(u) : pos[u]; }
    // st becomes 1 when u comes after v (the edge is charged to v), else 0;
    // with coarse ranks only the equal-class edges load u's position, all
    // of a thread's at once
    template <int EPT>
    __device__ __forceinline__ void resolve(const int (&jj)[EPT], const int (&uu)[EPT], int (&st)[EPT]) const {
        if (cb) {
            bool tie[EPT];
            int pu[EPT];
#pragma unroll
            for (int e = 0; e < EPT; e++)
                tie[e] = jj[e] >= 0 && st[e] == (int)((unsigned int)spos[jj[e]] >> CR_POS_BITS);
#pragma unroll
            for (int e = 0; e < EPT; e++) pu[e] = tie[e] ? pos[uu[e]] : 0;
#pragma unroll
            for (int e = 0; e < EPT; e++) {
                if (jj[e] < 0) continue;
                const unsigned int sv = (unsigned int)spos[jj[e]];
                st[e] = tie[e] ? (pu[e] > (int)(sv & ((1u << CR_POS_BITS) - 1)) ? 1 : 0)
                               : (st[e] > (int)(sv >> CR_POS_BITS) ? 1 : 0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < EPT; e++)
                if (jj[e] >= 0) st[e] = st[e] > spos[jj[e]] ? 1 : 0;
        }
    }
    __device__ __forceinline__ bool edge(int, int, int later, int, unsigned int) const { return later != 0; }
    __device__ __forceinline__ void flush_chunk() {}
};

__global__ __launch_bounds__(SORT_BLK) void k_sweep_sort(SweepArgs a) {
    __shared__ SweepLds<SORT_CH> s;
    __shared__ int spos[SORT_CH];
    SortEdgeOp op{a.pos, a.cb, a.ctl, spos};
    sweep_chunks<SORT_BLK, SORT_CH, 1>(a.K, a.E, a.iv, a.ie, a.ir, a.cfirst, a.clast, a.adj, a.inc, op, s, blockIdx.x,
                                    gridDim.x, nullptr, nullptr);
}

// =============================================================== SEQ
// One block runs the n single-vertex steps of the sequential load ordering.
// prio (load + current degree) lives in LDS; a peeled vertex gets the key
// 0xFFFFFFFF.  Each step: block argmin of (prio, id), record, decrement the
// neighbours still present.
__global__ __launch_bounds__(SEQ_BLK) void k_seq_order(int n, const int* __restrict__ off,
                                                       const int* __restrict__ adj, const int* __restrict__ load,
                                                       int* __restrict__ order, int* __restrict__ rnd,
                                                       int* __restrict__ inc, const int* __restrict__ perm,
                                                       const int* __restrict__ iperm) {
    constexpr int PER = (SEQ_MAX_N + SEQ_BLK - 1) / SEQ_BLK;
    extern __shared__ unsigned int sprio[];
    __shared__ unsigned long long shk[SEQ_BLK / WAVE];
    __shared__ int s_win;
    // ties go to the smallest caller id (the internal id unless hub-ordered)
    int cid[PER];
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int v = (int)threadIdx.x + k * SEQ_BLK;
        cid[k] = v < n ? (perm ? perm[v] : v) : 0;
        if (v < n) sprio[v] = (unsigned int)(load[v] + (off[v + 1] - off[v]));
    }
    __syncthreads();
    for (int j = 0; j < n; j++) {
        unsigned long long best = ~0ull;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int v = (int)threadIdx.x + k * SEQ_BLK;
            if (v < n) {
                const unsigned long long key = ((unsigned long long)sprio[v] << 32) | (unsigned int)cid[k];
                best = key < best ? key : best;
            }
        }
        best = block_min<SEQ_BLK>(best, shk);
        if (threadIdx.x == 0) {
            const int c = (int)(best & 0xFFFFFFFFull);
            const int w = iperm ? iperm[c] : c;
            order[j] = w;
            rnd[w] = j;
            inc[w] = (int)sprio[w] - load[w];
            sprio[w] = 0xFFFFFFFFu;
            s_win = w;
        }
        __syncthreads();
        const int a0 = off[s_win], a1 = off[s_win + 1];
        for (int e = a0 + threadIdx.x; e < a1; e += SEQ_BLK) {
            const int u = adj[e] & ADJ_ID_MASK;
            if (sprio[u] != 0xFFFFFFFFu) sprio[u] -= 1;
        }
        __syncthreads();
    }
}

// ======================================================== Algorithm 3
// A[i] = charge of the vertex at position i; per-tile sums.
__global__ __launch_bounds__(SCAN_BLK) void k_gather_A(int n, const int* __restrict__ order,
                                                       const int* __restrict__ inc, int* __restrict__ A,
                                                       long long* __restrict__ tile_sum) {
    __shared__ long long sh[SCAN_BLK / WAVE];
    long long base = (long long)blockIdx.x * SCAN_TILE;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k * SCAN_BLK + threadIdx.x;
        if (i < n) {
            int x = inc[order[i]];
            A[i] = x;
            s += x;
        }
    }
    s = block_sum<SCAN_BLK>(s, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// One block: suffix offsets of tiles, off[b] = sum of tiles after b.
__global__ __launch_bounds__(1024) void k_suffix_top(const long long* __restrict__ tile_sum,
                                                     long long* __restrict__ tile_off, int ntiles) {
    __shared__ long long sh[1024 / WAVE];
    long long carry = 0;
    // walk tiles from the end; reversed index r = ntiles-1-b
    for (int base = 0; base < ntiles; base += 1024) {
        int rr = base + threadIdx.x;
        int b = ntiles - 1 - rr;
        long long v = rr < ntiles ? tile_sum[b] : 0;
        long long tot;
        long long ex = block_excl_scan<1024>(v, &tot, sh);
        if (rr < ntiles) tile_off[b] = carry + ex;
        carry += tot;
    }
}

struct Cand {
    long long e, v, i;
};

// a better than b: strictly denser, or equally dense with a smaller index
__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
    long long l = a.e * b.v, r = b.e * a.v;
    return l > r || (l == r && a.i < b.i);
}

__device__ __forceinline__ Cand cand_shfl(const Cand& c, int o) {
    return Cand{__shfl_xor(c.e, o, WAVE), __shfl_xor(c.v, o, WAVE), __shfl_xor(c.i, o, WAVE)};
}

template <int BLK>
__device__ __forceinline__ Cand block_best(Cand c, Cand* sh) {
    constexpr int NW = BLK / WAVE;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        Cand w = cand_shfl(c, o);
        if (cand_better(w, c)) c = w;
    }
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) sh[wid] = c;
    __syncthreads();
    Cand b = sh[0];
#pragma unroll
    for (int w = 1; w < NW; w++)
        if (cand_better(sh[w], b)) b = sh[w];
    __syncthreads();
    return b;
}

// Per tile: B[i] = (suffix of later tiles) + sum of A[j], j >= i in the tile;
// candidate i has (B[i], n - i); the tile's densest, ties to smallest i.
// Thread t owns items [base + 16t, base + 16t + 16) (contiguous).
__global__ __launch_bounds__(SCAN_BLK) void k_suffix_argmax(int n, const int* __restrict__ A,
                                                            const long long* __restrict__ tile_off,
                                                            long long* __restrict__ tile_best) {
    __shared__ long long sh[SCAN_BLK / WAVE];
    __shared__ Cand shc[SCAN_BLK / WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    int x[SCAN_ITEMS];
    long long mysum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        long long i = base + k;
        x[k] = i < n ? A[i] : 0;
        mysum += x[k];
    }
    // suffix over threads: reverse-order exclusive scan
    long long tot;
    // exclusive scan in forward order gives sum of earlier threads; suffix = tot - excl - mine
    long long ex = block_excl_scan<SCAN_BLK>(mysum, &tot, sh);
    long long suffix_after = tile_off[blockIdx.x] + (tot - ex - mysum);
    Cand best{-1, 1, 0x7FFFFFFFFFFFFFFFll};
    long long run = suffix_after;
#pragma unroll
    for (int k = SCAN_ITEMS - 1; k >= 0; k--) {
        long long i = base + k;
        run += x[k];
        if (i < n) {
            Cand c{run, (long long)n - i, i};
            if (best.e < 0 || cand_better(c, best)) best = c;
        }
    }
    best = block_best<SCAN_BLK>(best, shc);
    if (threadIdx.x == 0) {
        tile_best[3 * blockIdx.x] = best.e;
        tile_best[3 * blockIdx.x + 1] = best.v;
        tile_best[3 * blockIdx.x + 2] = best.i;
    }
}

// One block: the iteration's densest suffix, history record, best update.
__global__ __launch_bounds__(1024) void k_iter_end(const long long* __restrict__ tile_best, int ntiles, Ctl* ctl,
                                                   long long* __restrict__ hist_e, long long* __restrict__ hist_v,
                                                   int* __restrict__ hist_i, unsigned long long* __restrict__ digest,
                                                   int* __restrict__ rounds, int* __restrict__ hist_w,
                                                   int* __restrict__ hist_lmax, int slot, int nrounds_static) {
    __shared__ Cand shc[1024 / WAVE];
    Cand best{-1, 1, 0x7FFFFFFFFFFFFFFFll};
    for (int b = threadIdx.x; b < ntiles; b += 1024) {
        Cand c{tile_best[3 * b], tile_best[3 * b + 1], tile_best[3 * b + 2]};
        if (c.e >= 0 && (best.e < 0 || cand_better(c, best))) best = c;
    }
    best = block_best<1024>(best, shc);
    if (threadIdx.x == 0) {
        hist_e[slot] = best.e;
        hist_v[slot] = best.v;
        hist_i[slot] = (int)best.i;
        digest[slot] = 0;
        hist_w[slot] = 0;
        hist_lmax[slot] = 0;
        rounds[slot] = nrounds_static > 0 ? nrounds_static : ctl->nrounds;
        const int it = ctl->iters_done + 1;
        ctl->iters_done = it;
        // strict improvement only (the input graph is the initial best)
        if (best.e * ctl->best_v > ctl->best_e * best.v) {
            ctl->best_e = best.e;
            ctl->best_v = best.v;
            ctl->best_iter = it;
            ctl->best_idx = best.i;
            ctl->improved = 1;
        } else {
            ctl->improved = 0;
        }
    }
}

// load += charge; digest of (caller id, round); snapshot of the order on
// improvement.
__global__ __launch_bounds__(256) void k_finalize(int n, int* __restrict__ load, const int* __restrict__ inc,
                                                  const int* __restrict__ rnd, const int* __restrict__ order,
                                                  int* __restrict__ best_order, const Ctl* ctl,
                                                  unsigned long long* __restrict__ digest_slot, int* __restrict__ w_slot,
                                                  int* __restrict__ lmax_slot, const int* __restrict__ perm) {
    __shared__ unsigned long long sh[256 / WAVE];
    __shared__ unsigned int shm[256 / WAVE];
    const bool improved = ctl->improved != 0;
    unsigned long long h = 0;
    unsigned int wmax = 0, lmax = 0;  // loads and charges are non-negative
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int c = inc[v];
        const int l = load[v] + c;
        load[v] = l;
        wmax = max(wmax, (unsigned int)c);
        lmax = max(lmax, (unsigned int)l);
        const int cv = perm ? perm[v] : v;  // the digest is over caller ids
        h += mix64(((unsigned long long)(unsigned int)cv << 32) | (unsigned long long)(unsigned int)rnd[v]);
        if (improved) best_order[v] = order[v];
    }
    h = block_sum<256>(h, sh);
    // block maxima as minima of the complements: one atomic per block
    const unsigned int bw = 0xFFFFFFFFu - block_min<256>(0xFFFFFFFFu - wmax, shm);
    const unsigned int bl = 0xFFFFFFFFu - block_min<256>(0xFFFFFFFFu - lmax, shm);
    if (threadIdx.x == 0) {
        atomicAdd(digest_slot, h);
        atomicMax(w_slot, (int)bw);
        atomicMax(lmax_slot, (int)bl);
    }
}

// =============================================================== BATCH
// Many independent graphs in one persistent launch.  Each block takes whole
// graphs from a work queue (largest first) and runs all of a graph's PEEL
// iterations with block barriers only.  The grid-wide round loop is for one
// large graph.  The per-round rule, same-round edge ownership and
// Algorithm 3 bookkeeping are the same as in the grid-wide path.  Because
// one block owns a graph, the alive list is compacted in id order with block
// scans alone, so each round's frontier comes out in ascending id and its
// positions follow from one running count.
template <int SLOTS>
struct DecTableT {
    int key[SLOTS];
    int cnt[SLOTS];
};

template <int CH>
struct BatchLds {
    SweepLds<CH> sw;
    DecTableT<2 * CH> dec;
};

template <int BLK, int SLOTS>
struct BatchPeelOp {
    const int* rnd;
    int* prio;
    int r;
    unsigned int lmin;
    int* err;
    DecTableT<SLOTS>* dec;
    __device__ void flag_error() { atomicAdd(err, 1); }
    __device__ __forceinline__ void stage_item(int, int) {}
    __device__ __forceinline__ int gather(int u) const { return rnd[u]; }
    template <int EPT>
    __device__ __forceinline__ void resolve(const int (&)[EPT], const int (&)[EPT], int (&)[EPT]) const {}
    __device__ __forceinline__ bool edge(int v, int u, int ru, int, unsigned int) {
        if (ru < 0) {
            unsigned int h = ((unsigned int)u * 0x9E3779B1u) >> (32 - __builtin_ctz(SLOTS));
#pragma unroll 1
            for (int probe = 0; probe < 64; probe++) {
                const int k = atomicCAS(&dec->key[h], DEC_EMPTY, u);
                if (k == DEC_EMPTY || k == u) {
                    atomicAdd(&dec->cnt[h], 1);
                    return true;
                }
                h = (h + 1) & (SLOTS - 1);
            }
            const int old = atomicSub(&prio[u], 1);
            lmin = min(lmin, (unsigned int)(old - 1));
            return true;
        }
        return ru == r && u > v;
    }
    __device__ __forceinline__ void flush_chunk() {
        constexpr int PER = SLOTS / BLK;
        lds_barrier();
        int key[PER], c[PER], old[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            key[k] = dec->key[threadIdx.x + k * BLK];
            c[k] = dec->cnt[threadIdx.x + k * BLK];
        }
#pragma unroll
        for (int k = 0; k < PER; k++)
            if (key[k] != DEC_EMPTY) old[k] = atomicSub(&prio[key[k]], c[k]);
#pragma unroll
        for (int k = 0; k < PER; k++) {
            if (key[k] != DEC_EMPTY) {
                lmin = min(lmin, (unsigned int)(old[k] - c[k]));
                dec->key[threadIdx.x + k * BLK] = DEC_EMPTY;
                dec->cnt[threadIdx.x + k * BLK] = 0;
            }
        }
    }
};

// One PEEL iteration of one graph by one block.
template <int BLK, int CH>
__device__ void batch_iteration(const BatchDesc& d, BatchLds<CH>& lds, int* err, const int slot) {
    constexpr int U = 4;
    constexpr int TILE = BLK * U;
    __shared__ unsigned long long sh64[BLK / WAVE];
    __shared__ unsigned int sh32[BLK / WAVE];
    __shared__ Cand shc[BLK / WAVE];
    __shared__ int s_improved;
    const int n = d.n;
    const long long q = d.eps_den, p = d.eps_num;
    // ---- init
    unsigned int lmin = 0xFFFFFFFFu;
    for (int v = threadIdx.x; v < n; v += BLK) {
        const int pv = d.load[v] + (d.off[v + 1] - d.off[v]);
        d.prio[v] = pv;
        d.rnd[v] = -1;
        d.inc[v] = 0;
        lmin = min(lmin, (unsigned int)pv);
    }
    unsigned int mn = block_min<BLK>(lmin, sh32);
    int Lc = n, next = 0, r = 0;
    // ---- rounds
    while (Lc > 0) {
        const int* __restrict__ Lin = (r & 1) ? d.L1 : d.L0;
        int* __restrict__ Lout = (r & 1) ? d.L0 : d.L1;
        const long long thr = ((q + p) * (long long)mn) / q;
        unsigned int smin = 0xFFFFFFFFu;
        int nfr = 0, nitem = 0, nsurv = 0;
        long long nedge = 0;
        for (int base = 0; base < Lc; base += TILE) {
            int u[U], pu[U], o0[U], o1[U];
#pragma unroll
            for (int k = 0; k < U; k++) {
                const int idx = base + (int)threadIdx.x * U + k;
                u[k] = idx < Lc ? ((r == 0) ? idx : Lin[idx]) : -1;
            }
#pragma unroll
            for (int k = 0; k < U; k++) pu[k] = u[k] >= 0 ? d.prio[u[k]] : 0;
#pragma unroll
            for (int k = 0; k < U; k++) {
                const bool fr = u[k] >= 0 && (long long)pu[k] <= thr;
                o0[k] = fr ? d.off[u[k]] : 0;
                o1[k] = fr ? d.off[u[k] + 1] : 0;
            }
            // counts [frontier:16][items:16][survivors:16] and edges
            unsigned long long cnt = 0, edg = 0;
#pragma unroll
            for (int k = 0; k < U; k++) {
                if (u[k] < 0) continue;
                if ((long long)pu[k] <= thr) {
                    cnt += 1ull;
                    if (o1[k] > o0[k]) {
                        cnt += 1ull << 16;
                        edg += (unsigned long long)(o1[k] - o0[k]);
                    }
                } else {
                    cnt += 1ull << 32;
                }
            }
            unsigned long long ctot, etot;
            unsigned long long cex = block_excl_scan<BLK>(cnt, &ctot, sh64);
            unsigned long long eex = block_excl_scan<BLK>(edg, &etot, sh64);
            int f = nfr + (int)(cex & 0xFFFF);
            int it = nitem + (int)((cex >> 16) & 0xFFFF);
            int sv = nsurv + (int)((cex >> 32) & 0xFFFF);
            long long ed = nedge + (long long)eex;
#pragma unroll
            for (int k = 0; k < U; k++) {
                if (u[k] < 0) continue;
                if ((long long)pu[k] <= thr) {
                    d.pos[u[k]] = next + f++;
                    d.rnd[u[k]] = r;
                    const int dg = o1[k] - o0[k];
                    if (dg > 0) {
                        d.iv[it] = u[k];
                        d.ie[it] = (int)ed;
                        d.ir[it] = o0[k] - (int)ed;
                        mark_chunks<CH>(ed, ed + dg, it, d.cfirst, d.clast);
                        it++;
                        ed += dg;
                    }
                } else {
                    Lout[sv++] = u[k];
                    smin = min(smin, (unsigned int)pu[k]);
                }
            }
            nfr += (int)(ctot & 0xFFFF);
            nitem += (int)((ctot >> 16) & 0xFFFF);
            nsurv += (int)((ctot >> 32) & 0xFFFF);
            nedge += (long long)etot;
        }
        __syncthreads();
        BatchPeelOp<BLK, 2 * CH> op{d.rnd, d.prio, r, smin, err, &lds.dec};
        sweep_chunks<BLK, CH, 1>(nitem, nedge, d.iv, d.ie, d.ir, d.cfirst, d.clast, d.adj, d.inc, op, lds.sw, 0, 1,
                              nullptr, nullptr);
        __syncthreads();
        mn = block_min<BLK>(op.lmin, sh32);
        if (nsurv >= Lc) {  // every round peels the minimum vertex
            if (threadIdx.x == 0) atomicAdd(err, 1);
            break;
        }
        next += nfr;
        Lc = nsurv;
        r++;
    }
    // ---- Algorithm 3: A[pos] = charge, densest suffix (ties to the smallest index)
    for (int v = threadIdx.x; v < n; v += BLK) d.A[d.pos[v]] = d.inc[v];
    __syncthreads();
    long long carry = 0;
    Cand best{-1, 1, 0x7FFFFFFFFFFFFFFFll};
    for (int t0 = ((n - 1) / TILE) * TILE; t0 >= 0; t0 -= TILE) {
        const int b0 = t0 + (int)threadIdx.x * U;
        int x[U];
        long long mine = 0;
#pragma unroll
        for (int k = 0; k < U; k++) {
            x[k] = b0 + k < n ? d.A[b0 + k] : 0;
            mine += x[k];
        }
        long long tot;
        const long long ex = block_excl_scan<BLK>(mine, &tot, (long long*)sh64);
        long long run = carry + (tot - ex - mine);
        Cand c{-1, 1, 0x7FFFFFFFFFFFFFFFll};
#pragma unroll
        for (int k = U - 1; k >= 0; k--) {
            const int i = b0 + k;
            run += x[k];
            if (i < n) {
                Cand cc{run, (long long)(n - i), (long long)i};
                if (c.e < 0 || cand_better(cc, c)) c = cc;
            }
        }
        c = block_best<BLK>(c, shc);
        if (c.e >= 0 && (best.e < 0 || cand_better(c, best))) best = c;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        d.hist_e[slot] = best.e;
        d.hist_v[slot] = best.v;
        d.hist_i[slot] = (int)best.i;
        d.rounds[slot] = r;
        long long* bs = d.best;
        const int improved = best.e * bs[1] > bs[0] * best.v;
        if (improved) {
            bs[0] = best.e;
            bs[1] = best.v;
            bs[2] = slot + 1;
            bs[3] = best.i;
        }
        s_improved = improved;
    }
    __syncthreads();
    const bool improved = s_improved != 0;
    unsigned long long h = 0;
    for (int v = threadIdx.x; v < n; v += BLK) {
        d.load[v] += d.inc[v];
        h += mix64(((unsigned long long)(unsigned int)v << 32) | (unsigned long long)(unsigned int)d.rnd[v]);
        if (improved) d.best_pos[v] = d.pos[v];
    }
    h = block_sum<BLK>(h, sh64);
    if (threadIdx.x == 0) {
        d.digest[slot] = h;
        d.state[4] = slot + 1;
    }
    __syncthreads();
}

template <int BLK, int CH>
__global__ __launch_bounds__(BLK) void k_batch_peel(const BatchDesc* __restrict__ descs, const int* __restrict__ order,
                                                    int count, unsigned int* queue, int* err) {
    __shared__ BatchLds<CH> lds;
    __shared__ int s_g;
    for (int i = threadIdx.x; i < 2 * CH; i += BLK) {
        lds.dec.key[i] = DEC_EMPTY;
        lds.dec.cnt[i] = 0;
    }
    while (true) {
        if (threadIdx.x == 0) s_g = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int gi = s_g;
        __syncthreads();
        if (gi >= count) break;
        const BatchDesc d = descs[order[gi]];
        const int s0 = d.state[4];
        if (s0 + d.T > d.t_cap) {  // the host checks this; never index past the history
            if (threadIdx.x == 0) atomicAdd(err, 1);
            continue;
        }
        for (int t = 0; t < d.T; t++) batch_iteration<BLK, CH>(d, lds, err, s0 + t);
    }
}

__global__ void k_batch_reset(BatchDesc* descs, int count) {
    // loads 0, best = the input graph, history empty
    for (int g = blockIdx.x; g < count; g += gridDim.x) {
        const BatchDesc d = descs[g];
        for (int v = threadIdx.x; v < d.n; v += blockDim.x) d.load[v] = 0;
        if (threadIdx.x == 0) {
            d.best[0] = d.nnz / 2;
            d.best[1] = d.n;
            d.best[2] = 0;
            d.best[3] = 0;
            d.state[4] = 0;
            d.state[5] = 0;
        }
    }
}

// =============================================================== SERVE
// Continuous batching: one persistent kernel serves a request stream.  The
// host publishes request descriptors into a ring in pinned host memory and
// raises `tail`.  An idle block claims the next request with a CAS on a
// device counter and runs all of its iterations (the same per-graph
// iteration as the batch kernel, so results equal those of a lone run).
// It then signals completion through the slot's `done` word.  Requests that
// arrive while others run start as soon as a block is free.  Every block
// leaves once the host raises `shutdown` and the queue is drained, after
// `idle_ticks` of waiting with nothing to claim, or after `max_ticks` in
// total (wall clock at 100 MHz), so the grid always drains.
template <int BLK, int CH>
__global__ __launch_bounds__(BLK) void k_serve(ServeHostCtl* hc, ServeSlot* ring, int ring_size,
                                               unsigned long long* dhead, int* err, unsigned long long idle_ticks,
                                               unsigned long long max_ticks) {
    __shared__ BatchLds<CH> lds;
    __shared__ long long s_claim;
    __shared__ BatchDesc s_desc;
    for (int i = threadIdx.x; i < 2 * CH; i += BLK) {
        lds.dec.key[i] = DEC_EMPTY;
        lds.dec.cnt[i] = 0;
    }
    const unsigned long long t_start = wall_clock64();
    while (true) {
        if (threadIdx.x == 0) {
            long long claim = -1;
            const unsigned long long idle_from = wall_clock64();
            while (true) {
                const unsigned long long tail =
                    __hip_atomic_load(&hc->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                const unsigned long long h = __hip_atomic_load(dhead, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < tail) {
                    if (atomicCAS(dhead, h, h + 1) == h) {
                        claim = (long long)h;
                        break;
                    }
                    continue;
                }
                if (__hip_atomic_load(&hc->shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                const unsigned long long now = wall_clock64();
                if (now - idle_from > idle_ticks || now - t_start > max_ticks) break;
                __builtin_amdgcn_s_sleep(127);
            }
            s_claim = claim;
        }
        __syncthreads();
        const long long claim = s_claim;
        if (claim < 0) break;
        ServeSlot* sl = &ring[claim % ring_size];
        {
            // the descriptor sits in host memory: read it once, into LDS
            const int* src = reinterpret_cast<const int*>(&sl->d);
            int* dst = reinterpret_cast<int*>(&s_desc);
            for (int w = threadIdx.x; w < (int)(sizeof(BatchDesc) / 4); w += BLK)
                dst[w] = __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
        const BatchDesc d = s_desc;
        for (int v = threadIdx.x; v < d.n; v += BLK) d.load[v] = 0;
        if (threadIdx.x == 0) {
            d.best[0] = d.nnz / 2;
            d.best[1] = d.n;
            d.best[2] = 0;
            d.best[3] = 0;
            d.state[4] = 0;
        }
        __syncthreads();
        const int T = d.T < d.t_cap ? d.T : d.t_cap;
        for (int t = 0; t < T; t++) batch_iteration<BLK, CH>(d, lds, err, t);
        if (threadIdx.x == 0) {
            d.state[4] = T;
            // results are in device memory: write the L2 back before the host
            // sees the flag and copies them out
            __threadfence_system();
            __hip_atomic_store(&sl->done, (unsigned long long)claim + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
    }
}

// ================================================================= launchers
namespace {
inline int grid_for(long long n, int blk, int cap = 4096) {
    long long g = (n + blk - 1) / blk;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
}  // namespace

int ctl_bytes() { return (int)sizeof(Ctl); }

int peel_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_peel_rounds<false, false>), PEEL_BLK, 0) !=
        hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_zero_ctl(const GraphDev& g, hipStream_t s) {
    const int words = (int)(sizeof(Ctl) / sizeof(int));
    k_fill_i32<<<1, 256, 0, s>>>(reinterpret_cast<int*>(g.ctl), 0, words);
    return hipGetLastError();
}

hipError_t launch_check_offsets(const GraphDev& g, hipStream_t s) {
    k_check_offsets<<<grid_for(g.n, 256), 256, 0, s>>>(g.n, g.nnz, g.off, g.ctl);
    return hipGetLastError();
}

hipError_t launch_check_range(const GraphDev& g, hipStream_t s) {
    if (g.nnz > 0) k_check_range<<<grid_for(g.nnz, 256, 16384), 256, 0, s>>>(g.n, g.nnz, g.adj, g.ctl);
    return hipGetLastError();
}

hipError_t launch_check_rows(const GraphDev& g, hipStream_t s) {
    // needs n, nnz, off, adj and ctl only; offsets and entries already checked
    if (g.nnz == 0) return hipSuccess;
    const long long nchunks = (g.nnz + SORT_CH - 1) / SORT_CH;
    const int grid = (int)(nchunks < 8192 ? nchunks : 8192);
    k_check_rows<<<grid, SORT_BLK, 0, s>>>(g.n, g.nnz, g.off, g.adj, g.ctl);
    return hipGetLastError();
}

hipError_t launch_build_static_items(const GraphDev& g, hipStream_t s) {
    const int ntiles = ceil_div(g.n, SCAN_TILE);
    k_nonzero_flags<<<grid_for(g.n, 256), 256, 0, s>>>(g.n, g.off, g.A);
    k_scan_tile_sums<<<ntiles, SCAN_BLK, 0, s>>>(g.A, g.n, g.tile_sum);
    k_scan_top<<<1, 1024, 0, s>>>(g.tile_sum, ntiles, g.tile_off);
    // tile_off[0] receives the total after the scan of tile_sum in place; the
    // compaction reads the scanned tile_sum as its offsets
    k_compact_items<<<ntiles, SCAN_BLK, 0, s>>>(g.n, g.off, g.tile_sum, g.siv, g.sie, g.sir, g.scf, g.scl);
    return hipGetLastError();
}

// Degree sum of each owner range, written to rbase[j + 1]: block j sums its
// single ids (j, j + 2^sb, ... below bm.hub) and its lines above (line l
// covers ids bm.hub + [l 2^ls, (l + 1) 2^ls) and belongs to range l mod 2^sb).
__global__ __launch_bounds__(256) void k_bucket_cap(int n, const int* __restrict__ off, BktMap bm,
                                                    int* __restrict__ rbase) {
    __shared__ long long sh[256 / WAVE];
    const int j = blockIdx.x;
    const int sb = bm.sb;
    long long sum = 0;
    const int nh = min(n, bm.hub);
    for (int u = j + ((int)threadIdx.x << sb); u < nh; u += 256 << sb) sum += off[u + 1] - off[u];
    const long long rest = (long long)n - nh;
    const long long nlines = (rest + (1LL << bm.ls) - 1) >> bm.ls;
    for (long long l = j + ((long long)threadIdx.x << sb); l < nlines; l += 256LL << sb) {
        const long long v0 = nh + (l << bm.ls);
        const long long v1 = min((long long)n, v0 + (1LL << bm.ls));
        sum += off[v1] - off[v0];
    }
    sum = block_sum<256>(sum, sh);
    if (threadIdx.x == 0) rbase[j + 1] = (int)sum;
}

// Exclusive scan of the nr range sums into bucket starts (one block; nr <=
// BKT_MAX_NR = 2 * 1024).
__global__ __launch_bounds__(1024) void k_bucket_scan(int nr, int* __restrict__ rbase) {
    __shared__ int sh[1024 / WAVE];
    const int i0 = 2 * (int)threadIdx.x;
    const int a0 = i0 < nr ? rbase[i0 + 1] : 0;
    const int a1 = i0 + 1 < nr ? rbase[i0 + 2] : 0;
    int total;
    const int base = block_excl_scan<1024>(a0 + a1, &total, sh);
    if (i0 < nr) rbase[i0 + 1] = base + a0;
    if (i0 + 1 < nr) rbase[i0 + 2] = base + a0 + a1;
    if (threadIdx.x == 0) rbase[0] = 0;
}

hipError_t launch_bucket_bases(const GraphDev& g, hipStream_t s) {
    if (g.nr <= 0) return hipSuccess;
    k_bucket_cap<<<g.nr, 256, 0, s>>>(g.n, g.off, g.bm, g.rbase);
    k_bucket_scan<<<1, 1024, 0, s>>>(g.nr, g.rbase);
    return hipGetLastError();
}

// ============================================================ hub order
// Built once per graph.  Keys max_deg - degree sort the vertices by
// non-increasing degree; the radix sort is stable, so ties keep the caller's
// id order.
__global__ void k_hub_keys(int n, const int* __restrict__ off, int max_deg, int* __restrict__ key) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        key[v] = max_deg - (off[v + 1] - off[v]);
}

// perm = the sorted order; iperm its inverse; deg[i] = degree of internal i.
__global__ void k_hub_perm(int n, const int* __restrict__ order, const int* __restrict__ off, int* __restrict__ perm,
                           int* __restrict__ iperm, int* __restrict__ deg) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = order[i];
        perm[i] = v;
        iperm[v] = i;
        deg[i] = off[v + 1] - off[v];
    }
}

// off_h = exclusive prefix sums of deg (tile offsets already scanned in
// tile_off), off_h[n] = nnz.
__global__ __launch_bounds__(SCAN_BLK) void k_hub_offsets(int n, const int* __restrict__ deg,
                                                          const long long* __restrict__ tile_off,
                                                          int* __restrict__ off_h) {
    __shared__ int sh[SCAN_BLK / WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE;
    long long run = tile_off[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const long long i = base + k * SCAN_BLK + threadIdx.x;
        const int d = i < n ? deg[i] : 0;
        int tot;
        const int ex = block_excl_scan<SCAN_BLK>(d, &tot, sh);
        if (i < n) off_h[i] = (int)(run + ex);
        if (i == n - 1) off_h[n] = (int)(run + ex + d);
        run += tot;
    }
}

// The renumbered rows, edge-parallel over the new adjacency: a block takes
// SORT_CH consecutive entries, finds the rows holding the first and last by
// binary search, and each thread finds its entry's row inside that range.
// Entry x of internal row i is the caller's entry of row perm[i] at the same
// offset, renumbered, with bit 31 set when its caller id is above perm[i].
__global__ __launch_bounds__(SORT_BLK) void k_hub_adj(int n, long long nnz, const int* __restrict__ off,
                                                      const int* __restrict__ adj, const int* __restrict__ off_h,
                                                      const int* __restrict__ perm, const int* __restrict__ iperm,
                                                      int* __restrict__ adj_h) {
    __shared__ int s_k[2];
    const long long nchunks = (nnz + SORT_CH - 1) / SORT_CH;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long x0 = c * SORT_CH, x1 = min(nnz, x0 + SORT_CH);
        if (threadIdx.x < 2) s_k[threadIdx.x] = row_of_entry(off_h, 0, n - 1, threadIdx.x == 0 ? x0 : x1 - 1);
        __syncthreads();
        const int k0 = s_k[0], k1 = s_k[1];
        for (long long x = x0 + threadIdx.x; x < x1; x += SORT_BLK) {
            const int i = row_of_entry(off_h, k0, k1, x);
            const int v = perm[i];
            const int u = adj[off[v] + (int)(x - off_h[i])];
            adj_h[x] = iperm[u] | (u > v ? (int)~ADJ_ID_MASK : 0);
        }
        __syncthreads();  // s_k is rewritten for the next chunk
    }
}

static hipError_t enqueue_radix(const GraphDev& g, const int* key_src, int passes, hipStream_t s);

hipError_t launch_hub_order(const GraphDev& g, int max_deg, int* off_h, int* adj_h, int* perm, int* iperm,
                            hipStream_t s) {
    GraphDev d = g;  // the sort below must see the caller's ids
    d.perm = nullptr;
    d.iperm = nullptr;
    int bits = 0;
    while (bits < 31 && (1LL << bits) <= (long long)max_deg) bits++;
    const int passes = bits < 8 ? 1 : (bits + 7) / 8;
    k_hub_keys<<<grid_for(d.n, 256, 4096), 256, 0, s>>>(d.n, d.off, max_deg, d.load);
    hipError_t e = enqueue_radix(d, d.load, passes, s);
    if (e != hipSuccess) return e;
    k_hub_perm<<<grid_for(d.n, 256, 4096), 256, 0, s>>>(d.n, d.order, d.off, perm, iperm, d.A);
    const int ntiles = ceil_div(d.n, SCAN_TILE);
    k_scan_tile_sums<<<ntiles, SCAN_BLK, 0, s>>>(d.A, d.n, d.tile_sum);
    k_scan_top<<<1, 1024, 0, s>>>(d.tile_sum, ntiles, d.tile_off);
    k_hub_offsets<<<ntiles, SCAN_BLK, 0, s>>>(d.n, d.A, d.tile_sum, off_h);
    if (d.nnz > 0) {
        const long long nchunks = (d.nnz + SORT_CH - 1) / SORT_CH;
        const int grid = (int)(nchunks < 8192 ? nchunks : 8192);
        k_hub_adj<<<grid, SORT_BLK, 0, s>>>(d.n, d.nnz, d.off, d.adj, off_h, perm, iperm, adj_h);
    }
    return hipGetLastError();
}

hipError_t launch_reset_state(const GraphDev& g, hipStream_t s) {
    k_fill_i32<<<grid_for(g.n, 256), 256, 0, s>>>(g.load, 0, g.n);
    k_ctl_reset<<<1, 64, 0, s>>>(g.ctl, g.nnz / 2, g.n);
    return hipGetLastError();
}

// Stable LSD radix sort of the n vertex ids by key_src[v] over `passes`
// 8-bit digits; the sorted ids land in g.order.
// One stable LSD pass: keys kin (values vin, or the index when null) by the
// 8-bit digit at `shift` into kout (may be null) / vout.
static void enqueue_radix_pass(const GraphDev& g, const int* kin, const int* vin, int* kout, int* vout, int shift,
                               const int* gate, hipStream_t s) {
    const int rt = ceil_div(g.n, RTILE);
    const int total = RBINS * rt;
    const int st = ceil_div(total, SCAN_TILE);
    k_radix_hist<<<rt, RBLK, 0, s>>>(kin, g.n, shift, g.rhist, rt, gate);
    k_rscan_tiles<<<st, SCAN_BLK, 0, s>>>(g.rhist, total, g.tile_off, gate);
    k_rscan_top<<<1, 1024, 0, s>>>(g.tile_off, st, gate);
    k_rscan_apply<<<st, SCAN_BLK, 0, s>>>(g.rhist, total, g.tile_off, gate);
    k_radix_scatter<<<rt, RBLK, 0, s>>>(kin, vin, kout, vout, g.n, shift, g.rhist, rt, gate);
}

// out[i] = src[idx[i]]
__global__ void k_gather_keys(int n, const int* __restrict__ idx, const int* __restrict__ src, int* __restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = src[idx[i]];
}

// First pass input of a stable sort whose ties go to the smaller caller id:
// the internal ids in caller-id order (iperm) with their keys, under hub
// order; the identity otherwise.  The gathered keys go to g.kB, which the
// first pass only reads.
static void radix_first_input(const GraphDev& g, const int* key_src, const int** kin, const int** vin,
                              hipStream_t s) {
    *kin = key_src;
    *vin = nullptr;
    if (g.iperm) {
        k_gather_keys<<<grid_for(g.n, 256, 4096), 256, 0, s>>>(g.n, g.iperm, key_src, g.kB);
        *kin = g.kB;
        *vin = g.iperm;
    }
}

static hipError_t enqueue_radix(const GraphDev& g, const int* key_src, int passes, hipStream_t s) {
    const int *k0, *v0;
    radix_first_input(g, key_src, &k0, &v0, s);
    for (int p = 0; p < passes; p++) {
        const int* kin = p == 0 ? k0 : ((p - 1) & 1 ? g.kB : g.kA);
        const int* vin = p == 0 ? v0 : ((p - 1) & 1 ? g.vB : g.vA);
        int* kout = p == passes - 1 ? nullptr : (p & 1 ? g.kB : g.kA);
        int* vout = p == passes - 1 ? g.order : (p & 1 ? g.vB : g.vA);
        enqueue_radix_pass(g, kin, vin, kout, vout, 8 * p, nullptr, s);
    }
    return hipGetLastError();
}

// The order by (round, id) after a near-list round loop, or any round loop
// under hub order (ids are the caller's): a stable sort of the vertices by
// round.  Rounds number at most n.  Up to 2^16 vertices two passes
// suffice; above, the first two passes already leave their result in the
// order array, and the two upper passes (order -> vA -> order) skip
// themselves when the iteration had at most 2^16 rounds, as it nearly always
// has.
static hipError_t enqueue_sort_by_round(const GraphDev& g, hipStream_t s) {
    const int *k0, *v0;
    radix_first_input(g, g.rnd, &k0, &v0, s);
    if (g.n <= 256) {
        enqueue_radix_pass(g, k0, v0, nullptr, g.order, 0, nullptr, s);
    } else if (g.n <= (1 << 16)) {
        enqueue_radix_pass(g, k0, v0, g.kA, g.vA, 0, nullptr, s);
        enqueue_radix_pass(g, g.kA, g.vA, nullptr, g.order, 8, nullptr, s);
    } else {
        const int* gate = &g.ctl->nrounds;
        enqueue_radix_pass(g, k0, v0, g.kA, g.vA, 0, nullptr, s);
        enqueue_radix_pass(g, g.kA, g.vA, g.kB, g.order, 8, nullptr, s);
        enqueue_radix_pass(g, g.kB, g.order, g.kA, g.vA, 16, gate, s);
        enqueue_radix_pass(g, g.kA, g.vA, nullptr, g.order, 24, gate, s);
    }
    return hipGetLastError();
}

// Algorithm 3 on the order in g.order with charges in g.inc, then the
// history record, best update, load update and digest.
static hipError_t enqueue_alg3(const GraphDev& g, int slot, int nrounds_static, hipStream_t s) {
    const int ntiles = ceil_div(g.n, SCAN_TILE);
    k_gather_A<<<ntiles, SCAN_BLK, 0, s>>>(g.n, g.order, g.inc, g.A, g.tile_sum);
    k_suffix_top<<<1, 1024, 0, s>>>(g.tile_sum, g.tile_off, ntiles);
    k_suffix_argmax<<<ntiles, SCAN_BLK, 0, s>>>(g.n, g.A, g.tile_off, g.tile_best);
    k_iter_end<<<1, 1024, 0, s>>>(g.tile_best, ntiles, g.ctl, g.hist_e, g.hist_v, g.hist_i, g.digest, g.rounds,
                                  g.hist_w, g.hist_lmax, slot, nrounds_static);
    k_finalize<<<grid_for(g.n, 256, 2048), 256, 0, s>>>(g.n, g.load, g.inc, g.rnd, g.order, g.best_order, g.ctl,
                                                        g.digest + slot, g.hist_w + slot, g.hist_lmax + slot, g.perm);
    return hipGetLastError();
}

hipError_t enqueue_iter_peel(const GraphDev& g, int slot, int eps_num, int eps_den, int peel_grid,
                             long long bkt_min_e, long long coarse_min_e, int mono, int near, hipStream_t s,
                             hipEvent_t ev_a, hipEvent_t ev_b) {
    k_iter_begin<<<1, 256, 0, s>>>(g.ctl, g.gsync, g.bfill, g.nr);
    k_peel_init<<<grid_for(g.n, 256, 2048), 256, 0, s>>>(g.n, g.off, g.load, g.prio, g.rnd, g.inc, g.st2, g.ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PeelArgs a{};
    a.n = g.n;
    a.eps_num = eps_num;
    a.eps_den = eps_den;
    a.off = g.off;
    a.adj = g.adj;
    a.prio = g.prio;
    a.rnd = g.rnd;
    a.inc = g.inc;
    a.L0 = g.L0;
    a.L1 = g.L1;
    a.iv0 = g.iv;
    a.iv1 = g.iv1;
    a.st2 = g.st2;
    a.ie = g.ie;
    a.ir = g.ir;
    a.cfirst = g.cfirst;
    a.clast = g.clast;
    a.ctl = g.ctl;
    a.gs = g.gsync;
    a.bkt = g.bkt;
    a.bfill = g.bfill;
    a.rshift = g.rshift;
    a.narrow = g.narrow;
    a.bm = g.bm;
    a.rbase = g.rbase;
    a.nr = g.nr;
    a.bkt_min_e = bkt_min_e;
    a.coarse_min_e = coarse_min_e;
    a.seg = g.seg;
    a.order = g.order;
    a.rmin = g.rmin;
    a.N0 = g.N0;
    a.N1 = g.N1;
    a.X0 = g.X0;
    a.X1 = g.X1;
    a.segF = g.segF;
    a.segN = g.segN;
    a.near_num = NEAR_B_NUM;
    a.near_den = NEAR_B_DEN;
    a.near_add = NEAR_B_ADD;
    a.hub = g.perm ? 1 : 0;
    // one segment per thread of a block (segment tables hold PEEL_BLK entries)
    if (peel_grid > (near ? NEAR_BLK : PEEL_BLK)) return hipErrorInvalidValue;
    void* args[] = {&a};
    if (ev_a && (e = hipEventRecord(ev_a, s)) != hipSuccess) return e;
    const void* kern = near ? (mono ? reinterpret_cast<const void*>(k_peel_rounds_near<true>)
                                    : reinterpret_cast<const void*>(k_peel_rounds_near<false>))
                            : (mono ? (a.hub ? reinterpret_cast<const void*>(k_peel_rounds<true, true>)
                                             : reinterpret_cast<const void*>(k_peel_rounds<true, false>))
                                    : (a.hub ? reinterpret_cast<const void*>(k_peel_rounds<false, true>)
                                             : reinterpret_cast<const void*>(k_peel_rounds<false, false>)));
    e = hipLaunchCooperativeKernel(kern, dim3(peel_grid), dim3(near ? NEAR_BLK : PEEL_BLK), args, 0, s);
    if (e != hipSuccess) return e;
    if (ev_b && (e = hipEventRecord(ev_b, s)) != hipSuccess) return e;
    if (near || g.perm) {
        e = enqueue_sort_by_round(g, s);
        if (e != hipSuccess) return e;
    }
    // else the order is by round, ascending id inside a round (written by the
    // full-list round loop itself)
    return enqueue_alg3(g, slot, 0, s);
}

hipError_t enqueue_iter_sort(const GraphDev& g, int slot, int key_bits, int sort_grid, bool coarse, hipStream_t s,
                             hipEvent_t ev_a, hipEvent_t ev_b) {
    k_iter_begin<<<1, 64, 0, s>>>(g.ctl, nullptr, nullptr, 0);
    int passes = (key_bits + 7) / 8;
    if (passes < 1) passes = 1;
    hipError_t e = enqueue_radix(g, g.load, passes, s);
    if (e != hipSuccess) return e;
    coarse = coarse && g.nnz > 0;
    const int sshift = cr_shift(g.n);
    k_sort_pos<<<grid_for(g.n, 256, 2048), 256, 0, s>>>(g.n, g.order, g.rnd, g.inc, g.off,
                                                         coarse ? g.cr_samp : nullptr, sshift);
    if (coarse) {
        const int ntiles = (int)((((long long)g.n + (1LL << sshift) - 1) >> sshift) + CR_TILE - 1) / CR_TILE;
        k_coarse_tiles<<<ntiles, CR_TILE, 0, s>>>(g.n, sshift, g.cr_samp, g.cr_tsum);
        k_coarse_bounds<<<1, 1024, 0, s>>>(g.n, sshift, g.cr_samp, g.cr_tsum, g.cr_bounds);
        k_coarse_pack<<<grid_for((g.n + 7) / 8, 256, 2048), 256, 0, s>>>(g.n, g.rnd, g.cr_bounds, g.cb);
    }
    SweepArgs a{};
    a.K = g.n_items;
    a.E = g.nnz;
    a.iv = g.siv;
    a.ie = g.sie;
    a.ir = g.sir;
    a.cfirst = g.scf;
    a.clast = g.scl;
    a.off = g.off;
    a.adj = g.adj;
    a.inc = g.inc;
    a.pos = g.rnd;
    a.cb = coarse ? g.cb : nullptr;
    a.ctl = g.ctl;
    if (ev_a && (e = hipEventRecord(ev_a, s)) != hipSuccess) return e;
    if (g.nnz > 0) k_sweep_sort<<<sort_grid, SORT_BLK, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_b && (e = hipEventRecord(ev_b, s)) != hipSuccess) return e;
    if (e != hipSuccess) return e;
    return enqueue_alg3(g, slot, g.n, s);
}

hipError_t enqueue_iter_seq(const GraphDev& g, int slot, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
    k_iter_begin<<<1, 64, 0, s>>>(g.ctl, nullptr, nullptr, 0);
    hipError_t e;
    if (ev_a && (e = hipEventRecord(ev_a, s)) != hipSuccess) return e;
    k_seq_order<<<1, SEQ_BLK, sizeof(unsigned int) * (size_t)g.n, s>>>(g.n, g.off, g.adj, g.load, g.order, g.rnd,
                                                                          g.inc, g.perm, g.iperm);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_b && (e = hipEventRecord(ev_b, s)) != hipSuccess) return e;
    return enqueue_alg3(g, slot, g.n, s);
}


template <int BLK, int CH>
static hipError_t launch_batch_cfg(const BatchDesc* descs, const int* order, int count, unsigned int* queue, int* err,
                                   int blocks_per_cu, int num_cu, hipStream_t s) {
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_batch_peel<BLK, CH>),
                                                                BLK, 0);
    if (e != hipSuccess) return e;
    if (occ < 1) occ = 1;
    int per = blocks_per_cu < occ ? blocks_per_cu : occ;
    if (per < 1) per = 1;
    int grid = num_cu * per;
    if (grid > count) grid = count > 0 ? count : 1;
    k_batch_peel<BLK, CH><<<grid, BLK, 0, s>>>(descs, order, count, queue, err);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchDesc* descs, const int* order, int count, unsigned int* queue, int* err,
                        int cfg, int blocks_per_cu, int num_cu, hipStream_t s) {
    k_fill_i32<<<1, 64, 0, s>>>(reinterpret_cast<int*>(queue), 0, 1);
    switch (cfg) {
        case 0: return launch_batch_cfg<256, 1024>(descs, order, count, queue, err, blocks_per_cu, num_cu, s);
        case 1: return launch_batch_cfg<512, 2048>(descs, order, count, queue, err, blocks_per_cu, num_cu, s);
        default: return launch_batch_cfg<1024, 4096>(descs, order, count, queue, err, blocks_per_cu, num_cu, s);
    }
}

hipError_t launch_fill(int* p, int v, long long cnt, hipStream_t s) {
    k_fill_i32<<<grid_for(cnt, 256), 256, 0, s>>>(p, v, cnt);
    return hipGetLastError();
}

hipError_t launch_batch_reset(BatchDesc* descs, int count, hipStream_t s) {
    k_batch_reset<<<count < 2048 ? (count > 0 ? count : 1) : 2048, 256, 0, s>>>(descs, count);
    return hipGetLastError();
}


__global__ void k_set_u64(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) *p = v;
}

hipError_t launch_serve(ServeHostCtl* hc, ServeSlot* ring, int ring_size, unsigned long long* dhead,
                        unsigned long long head0, int* err, int cfg, int blocks_per_cu, int num_cu,
                        unsigned long long idle_ticks, unsigned long long max_ticks, hipStream_t s) {
    // the claim counter starts at the first unpublished ticket, in stream order
    // before the kernel
    k_set_u64<<<1, 64, 0, s>>>(dhead, head0);
    int grid = num_cu * (blocks_per_cu < 1 ? 1 : blocks_per_cu);
    switch (cfg) {
        case 0:
            k_serve<256, 1024><<<grid, 256, 0, s>>>(hc, ring, ring_size, dhead, err, idle_ticks, max_ticks);
            break;
        default:
            k_serve<512, 2048><<<grid, 512, 0, s>>>(hc, ring, ring_size, dhead, err, idle_ticks, max_ticks);
            break;
    }
    return hipGetLastError();
}

}  // namespace dsg
