// dsg_internal.h -- constants, kernel argument blocks and launchers shared by
// the kernels (dsg_kernels.hip) and the C ABI (dsg_api.hip).  Internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsg {

struct Ctl;
struct GridSync;

constexpr int PEEL_BLK = 1024;     // threads per block of the persistent round kernel
constexpr int PEEL_BLOCKS_PER_CU = 1;  // measured: two 512-thread blocks per CU are slower (more grid-sync arrivals)
constexpr int PEEL_CH = 4096;      // edges per coarse PEEL sweep chunk (items per chunk <= this)
constexpr int PEEL_MARK = 1024;    // PEEL chunk markers are written per 1024 edges; fine chunks are one marker,
                                   // coarse chunks PEEL_CH / PEEL_MARK markers
// a round sweeps coarse chunks when its frontier has at least this many edges (measured on R-MAT scale 22:
// about one coarse chunk per block of the grid)
constexpr long long PEEL_DEFAULT_COARSE_MIN_E = 1LL << 20;
constexpr int SORT_BLK = 512;      // threads per block of the SORT sweep
// edges per SORT sweep chunk: at 2048 a block's LDS is 40 KB and four blocks
// (8 waves per SIMD) share a CU; at 4096 (80 KB) only two did, and the SORT
// iteration on R-MAT scale 22 took 26% longer
constexpr int SORT_CH = 2048;
constexpr int MIN_CH = PEEL_MARK < SORT_CH ? PEEL_MARK : SORT_CH;  // finest chunk-marker granularity
constexpr int SEQ_BLK = 1024;      // threads of the single SEQ block
constexpr int SEQ_MAX_N = 16000;   // SEQ keeps n priorities in LDS (< 64 KB)
constexpr int PEEL_MAX_N = 1 << 26;  // frontier item counter has 26 bits
// Adjacency entries are indexed with int32, and a sweep chunk's edge
// positions (start + up to 4096) must stay below 2^31 as well.
constexpr long long MAX_NNZ = (1LL << 31) - (1LL << 16);
// Owner-bucketed decrements of the PEEL round loop.  Vertex ids are split
// into at most 2^sbits ranges (BktMap below: contiguous blocks of ids in the
// caller's order; under hub order the first BKT_HUB_IDS ids one by one and
// the others by 32-id lines, dealt round robin).  Inside its range a vertex
// has a local id below 2^lbits (lbits <= BKT_MAX_SHIFT, so a range's
// counters fit a dense LDS histogram).
// At most BKT_MAX_NR ranges, which covers every graph the PEEL path accepts
// (n < 2^26).  Rounds whose frontier has at least the threshold's edges take
// the bucketed path.
constexpr int BKT_MAX_SHIFT = 15;
constexpr int BKT_MAX_NR = 2048;
constexpr int BKT_LINE = 5;  // 32 ids per line
constexpr int BKT_HUB_IDS = 1 << 16;  // dealt singly; a multiple of 32 * BKT_MAX_NR
// Narrow bucket apply (16-bit counters, 2^16 local ids per range): under hub
// order when n needs at least 2^BKT_NARROW_MIN_SB such ranges and every
// vertex past the hub ids has degree below 2^16.
constexpr int BKT_NARROW_SHIFT = 16;
constexpr int BKT_NARROW_MIN_SB = 8;
static_assert(BKT_HUB_IDS % ((1 << BKT_LINE) * BKT_MAX_NR) == 0, "hub ids fill whole lines of every range");
constexpr int BKT_CNT_BITS = 12;  // bucket entry = local id << 12 | (count - 1); count <= PEEL_CH
constexpr long long BKT_DEFAULT_MIN_E = 1LL << 20;
// Under hub order the hubs' priorities share a few lines, and direct atomics
// on them contend, so rounds are bucketed from fewer frontier edges: 2^17
// took the 40M-vertex Chung-Lu graph's first 8 iterations from 51.8 to
// 49.8 ms each (2^14: 50.5, every round: 52.6).
constexpr long long BKT_HUB_DEFAULT_MIN_E = 1LL << 17;
// Near-list select (k_peel_rounds_near): the near bound is B = thr * 5/4 + 1
// at each full-list round.  The default from 2^23 vertices: on the 40M-vertex
// Chung-Lu graph its round loop takes 48.9 ms per iteration against 53.2 ms for
// the full-list select; on R-MAT scale 22 (2^22 vertices) it is slower (5.1
// against 4.6 ms).
constexpr int NEAR_B_NUM = 5;
constexpr int NEAR_B_DEN = 4;
constexpr int NEAR_B_ADD = 1;
constexpr int NEAR_DEFAULT_MIN_N = 1 << 23;
// SORT compares coarse ranks first once the position table (4n bytes) no
// longer fits an XCD's L2.  The 4-bit table (n/2 bytes) fits it up to 2^22
// vertices; above that both tables live in the MALL, where the 8x smaller
// one still wins (13.7% on the 40M-vertex Chung-Lu graph).  A staged word
// holds class << 28 | position, so n < 2^26.
constexpr int SORT_COARSE_MIN_N = 1 << 19;
constexpr int SORT_COARSE_MAX_N = (1 << 26) - 1;
static_assert((1 << BKT_CNT_BITS) >= 4096, "chunk-local counts must fit the entry's count field");
static_assert(BKT_MAX_SHIFT + BKT_CNT_BITS <= 32, "a bucket entry holds a local id and a count");
// Range layout for n vertices: about 256 ranges (one per block of the round
// loop) while a range's local ids fit 2^BKT_MAX_SHIFT, more above.  Returns
// false when the graph needs more than BKT_MAX_NR ranges (the bucketed path is
// then off).
inline bool bucket_params(long long n, int* lbits, int* sbits) {
    int cl = 0;
    while ((1LL << cl) < n) cl++;
    int l = cl - 8;
    if (l < BKT_LINE) l = BKT_LINE;
    if (l > BKT_MAX_SHIFT) l = BKT_MAX_SHIFT;
    const int sb = cl > l ? cl - l : 0;
    *lbits = l;
    *sbits = sb;
    return (1 << sb) <= BKT_MAX_NR;
}
static_assert(PEEL_MAX_N <= (1LL << (BKT_MAX_SHIFT + 11)) && (1 << 11) <= BKT_MAX_NR,
              "every graph the PEEL path accepts fits the bucketed path");

// Owner ranges of the bucketed decrements: 2^sb ranges.  The first `hub` ids
// are dealt one by one (u mod 2^sb), the rest by lines of 2^ls ids (line mod
// 2^sb).  In caller order a range is one contiguous block of ids (hub = 0,
// ls = the local id bits), so its priorities share few lines.  Under hub
// order the hubs come first and their decrements come from nearly every
// chunk: dealt singly (hub = BKT_HUB_IDS), then by 32-id lines (ls =
// BKT_LINE), they spread evenly over the ranges, where one block of them
// would overload a single range.  Local ids: the hub ids take the first
// hub >> sb slots of a range.
struct BktMap {
    int sb;   // log2 of the range count
    int ls;   // log2 of the line size
    int hub;  // ids dealt singly
    __device__ __forceinline__ int owner(int u) const {
        const int m = (1 << sb) - 1;
        return u < hub ? (u & m) : (((u - hub) >> ls) & m);
    }
    __device__ __forceinline__ int local(int u) const {
        if (u < hub) return u >> sb;
        const int w = u - hub;
        return (hub >> sb) + (((w >> (ls + sb)) << ls) | (w & ((1 << ls) - 1)));
    }
    __device__ __forceinline__ int global(int j, int li) const {
        const int h = hub >> sb;
        if (li < h) return (li << sb) | j;
        const int w = li - h;
        return hub + (((w >> ls) << (ls + sb)) | (j << ls) | (w & ((1 << ls) - 1)));
    }
};

struct PeelArgs {
    int n;
    int eps_num;
    int eps_den;
    int pad;
    const int* off;
    const int* adj;
    int* prio;
    int* rnd;
    int* inc;
    int* L0;
    int* L1;
    int* iv0;  // item vertices of even rounds
    int* iv1;  // item vertices of odd rounds
    unsigned int* st2;
    int* ie;
    int* ir;
    int* cfirst;
    int* clast;
    Ctl* ctl;
    GridSync* gs;
    int* bkt;              // owner buckets (nnz entries; range j's starts at rbase[j])
    unsigned int* bfill;   // per-range fill counters, zero between bucketed rounds
    const int* rbase;      // nr + 1 bucket starts: range j holds rbase[j + 1] - rbase[j] entries (its degree sum)
    int rshift;            // local id bits of a range
    BktMap bm;             // vertex -> (range, local id)
    int nr;                // ranges holding vertices; 0 = bucketed path off
    long long bkt_min_e;   // frontier edges from which a round is bucketed
    long long coarse_min_e;  // frontier edges from which a round sweeps coarse chunks
    int* seg;              // per block, by round parity: [2][alive start | alive len | frontier len][PEEL_BLK]
    int* order;            // order[position] = vertex, written round by round
    int* rmin;             // optional: rmin[r] = round r's priority bound thr (room for n rounds)
    // near-list select (k_peel_rounds_near)
    int* N0;               // near lists, by round parity
    int* N1;
    int* X0;               // crossing lists, by round parity of the round that reads them
    int* X1;
    int* segF;             // full-list segments, by parity: [2][start | len][PEEL_BLK]
    int* segN;             // near-list segments, by round parity: [2][start | len][PEEL_BLK]
    int near_num;          // near bound B = thr * near_num / near_den + near_add
    int near_den;
    int near_add;
    int hub;               // hub order: bit 31 of an entry tells whether the neighbour comes later in a round
    int narrow;            // bucket apply with 16-bit counters (rshift = BKT_NARROW_SHIFT)
};

struct SweepArgs {
    int K;
    int pad;
    long long E;
    const int* iv;
    const int* ie;
    const int* ir;
    const int* cfirst;
    const int* clast;
    const int* off;
    const int* adj;
    int* inc;
    const int* pos;
    const unsigned int* cb;  // SORT coarse ranks (4 bits per vertex) or null
    Ctl* ctl;
};

// Device pointers of one graph's state, carved from the workspace.
struct GraphDev {
    int n;
    long long nnz;
    const int* off;
    const int* adj;
    // hub order (null otherwise): internal vertex i is the caller's perm[i],
    // the caller's v is internal iperm[v]; off/adj are then the renumbered CSR
    const int* perm;
    const int* iperm;
    int* hub_off;    // hub order storage (carved when the flag is set)
    int* hub_adj;
    int* hub_perm;
    int* hub_iperm;
    Ctl* ctl;
    GridSync* gsync;
    int* load;
    int* prio;
    int* rnd;
    int* inc;
    int* order;
    int* best_order;
    int* kA;
    int* kB;
    int* vA;
    int* vB;
    int* L0;
    int* L1;
    int* iv;
    int* iv1;
    unsigned int* st2;
    int* ie;
    int* ir;
    int* siv;
    int* sie;
    int* sir;
    int* A;
    int* cfirst;
    int* clast;
    int* scf;
    int* scl;
    long long* tile_sum;
    long long* tile_off;
    long long* tile_best;
    int* rhist;
    long long* hist_e;
    long long* hist_v;
    int* hist_i;
    int* rounds;
    unsigned long long* digest;
    int* hist_w;     // per iteration: largest load increase (empirical width)
    int* hist_lmax;  // per iteration: largest load after it
    int* bkt;
    unsigned int* bfill;
    int* rbase;   // bucket starts per range (nr + 1), from the degree sums
    int rshift;   // local id bits of a range
    BktMap bm;
    int nr;
    int narrow;   // 16-bit bucket apply (hub order, see BKT_NARROW_SHIFT)
    unsigned int* cb;  // SORT coarse ranks
    int* cr_bounds;    // first position of each coarse class
    int* cr_samp;      // degrees at the sampled positions
    int* seg;          // PEEL alive-list segments (4 * PEEL_BLK ints)
    long long* cr_tsum;  // sampled degree mass per tile of 1024 samples
    int* rmin;         // optional, set by the caller for one run: per-round priority bound (n ints)
    int* N0;           // near-list select: near lists, crossing lists, segment tables
    int* N1;
    int* X0;
    int* X1;
    int* segF;
    int* segN;
    int n_items;  // vertices with degree > 0
    int max_deg;
};

// Hub order (DSG_HUB_ORDER): internal ids by non-increasing degree, ties by
// the caller's id.  Adjacency entries of the renumbered CSR carry the
// neighbour's internal id in bits 0-30 and, in bit 31, whether the
// neighbour's caller id is larger than the row vertex's.
constexpr int ADJ_ID_MASK = 0x7FFFFFFF;
// Builds perm, iperm and the renumbered CSR (off_h: n + 1, adj_h: nnz) from
// the caller's CSR in g.off / g.adj; uses g's radix and scan scratch and
// g.load as temporary keys.
hipError_t launch_hub_order(const GraphDev& g, int max_deg, int* off_h, int* adj_h, int* perm, int* iperm,
                            hipStream_t s);

// launchers (enqueue on `s`; return the first HIP error)
hipError_t launch_check_offsets(const GraphDev& g, hipStream_t s);
hipError_t launch_check_range(const GraphDev& g, hipStream_t s);
hipError_t launch_check_rows(const GraphDev& g, hipStream_t s);
hipError_t launch_build_static_items(const GraphDev& g, hipStream_t s);
hipError_t launch_bucket_bases(const GraphDev& g, hipStream_t s);
hipError_t launch_reset_state(const GraphDev& g, hipStream_t s);
hipError_t launch_zero_ctl(const GraphDev& g, hipStream_t s);

// One iteration; `slot` is the history index written by this iteration.
// ev_a / ev_b (may be null) are recorded on `s` right before and after the
// iteration's dominant kernel (PEEL round loop, SORT sweep, SEQ peel).
// mono: monotone round thresholds (Coreness by buckets); near: the near-list
// select (k_peel_rounds_near), which orders by round after the loop
hipError_t enqueue_iter_peel(const GraphDev& g, int slot, int eps_num, int eps_den, int peel_grid,
                             long long bkt_min_e, long long coarse_min_e, int mono, int near, hipStream_t s,
                             hipEvent_t ev_a, hipEvent_t ev_b);
hipError_t enqueue_iter_sort(const GraphDev& g, int slot, int key_bits, int sort_grid, bool coarse, hipStream_t s,
                             hipEvent_t ev_a, hipEvent_t ev_b);
hipError_t enqueue_iter_seq(const GraphDev& g, int slot, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b);

// One graph of a batch: its CSR and every per-graph array, carved from the
// batch workspace by the host.  state[4] = history slots used, state[5] =
// iterations done before the history was last cleared (always 0 here).
struct BatchDesc {
    int n;
    int T;
    int eps_num;
    int eps_den;
    long long nnz;
    const int* off;
    const int* adj;
    int* load;
    int* prio;
    int* rnd;
    int* inc;
    int* pos;
    int* L0;
    int* L1;
    int* iv;
    int* ie;
    int* ir;
    int* A;
    int* best_pos;
    int* cfirst;
    int* clast;
    long long* hist_e;
    long long* hist_v;
    int* hist_i;
    int* rounds;
    unsigned long long* digest;
    long long* best;  // edges, vertices, iteration, index
    int* state;       // [4] history slots used, [5] reserved
    int t_cap;
    int pad;
};

// cfg: 0 = 256 threads / 1024-edge chunks, 1 = 512 / 2048, 2 = 1024 / 4096
hipError_t launch_batch(const BatchDesc* descs, const int* order, int count, unsigned int* queue, int* err, int cfg,
                        int blocks_per_cu, int num_cu, hipStream_t s);
hipError_t launch_batch_reset(BatchDesc* descs, int count, hipStream_t s);
hipError_t launch_fill(int* p, int v, long long cnt, hipStream_t s);

// Serving: control block and request ring in pinned host memory.
struct ServeHostCtl {
    unsigned long long tail;  // requests published by the host
    unsigned long long pad0[7];
    unsigned int shutdown;    // host sets 1: blocks leave once the queue is drained
    unsigned int pad1[15];
};

struct ServeSlot {
    BatchDesc d;
    unsigned long long done;  // ticket + 1 once the result is in device memory
    unsigned long long pad[7];
};

// cfg 0 = 256 threads / 1024-edge chunks, otherwise 512 / 2048
hipError_t launch_serve(ServeHostCtl* hc, ServeSlot* ring, int ring_size, unsigned long long* dhead,
                        unsigned long long head0, int* err, int cfg, int blocks_per_cu, int num_cu,
                        unsigned long long idle_ticks, unsigned long long max_ticks, hipStream_t s);
constexpr int BATCH_MIN_CH = 1024;

int peel_blocks_per_cu();
int ctl_bytes();

}  // namespace dsg
