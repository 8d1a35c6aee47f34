// dsg_api.hip -- the C ABI of libdsg.so (declared in include/dsg.h).
//
// Host side only: argument checks, workspace carving, kernel sequencing and
// result fetches.  Every step of the algorithm runs in the kernels of
// dsg_kernels.hip.  The library allocates no device memory; all state lives
// in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dsg.h"
#include "dsg_device.h"
#include "dsg_internal.h"
#include "dsg_par.h"

using dsg::GraphDev;

// Static device scratch of dsg_par_run_noalloc.  Each GPU the library runs on
// holds its own copy from module load until the process ends.  In host code
// the name `scratch` is only a stand-in: its device address on each GPU comes
// from hipGetSymbolAddress (resolved once per device, at dsg_ctx_create) and
// only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[DSG_NOALLOC_SCRATCH_BYTES];

struct dsg_ctx {
    int device;
    hipStream_t stream;
    int num_cu;
    int peel_grid;
    int sort_grid;
};

struct dsg_graph {
    dsg_ctx* ctx;
    GraphDev d;
    char* ws;
    long long ws_bytes;
    int t_cap;
    int recorded;     // iterations recorded in the history
    int iters_done;   // iterations performed since the last reset (host mirror)
    long long load_bound;  // upper bound on every load (grows by max_degree per iteration; 0 after reset)
    int last_variant; // -1 = none yet
    hipEvent_t ev0, ev1;
    bool timed;
    bool ktime;                    // per-launch timing of the dominant kernel
    std::vector<hipEvent_t> kev;   // 2 events per timed launch
    int klaunches;                 // timed launches of the last dsg_run
    long long bkt_min_e;           // PEEL rounds with at least this many frontier edges use owner buckets
    long long coarse_min_e;        // ... and coarse sweep chunks; -1 = default
    int sort_coarse;               // SORT coarse ranks: -1 = by size, 0 = off, 1 = on
    int peel_select;               // PEEL select: -1 = by size, 0 = full list, 1 = near list
    // graph replay (dsg_set_graph_replay): the launches of one dsg_run are
    // captured on a private stream into a HIP graph, which later calls with
    // the same key replay on the context's stream
    bool replay;
    int replay_state;              // 1 = a run is captured, 0 = none yet, -1 = capture refused (eager from then on)
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    long long gkey[11];
};

struct dsg_batch {
    dsg_ctx* ctx;
    int count;
    int t_cap;
    std::vector<dsg::BatchDesc> hdesc;  // host copy of the descriptors
    std::vector<int> max_deg;
    std::vector<int> iters;             // iterations done per graph (host mirror)
    dsg::BatchDesc* ddesc;
    int* dorder;
    unsigned int* dqueue;
    int* derr;
    dsg::Ctl* dctl;                     // scratch control block for the CSR checks
    int cfg;
    int blocks_per_cu;
    hipEvent_t ev0, ev1;
    bool timed;
};

namespace {

thread_local std::string g_err;

// The device scratch of dsg_par_run_noalloc is `scratch` (file scope, above
// this namespace); its per-device addresses are kept here.
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[SCRATCH_MAX_DEVICES];
void* g_scratch_ptr[SCRATCH_MAX_DEVICES];
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES];

// Resolves the scratch address on `device` (which must be current), once.
void resolve_scratch(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
}

dsg_status fail(dsg_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

dsg_status hip_fail(hipError_t e, const char* where) {
    return fail(DSG_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define DSG_HIP(call, where)                                 \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return hip_fail(_e, (where));  \
    } while (0)

struct Layout {
    long long off[80];
    int count = 0;
    long long total = 0;
    long long add(long long bytes) {
        long long at = total;
        off[count++] = at;
        total += (bytes + 255) / 256 * 256;
        return at;
    }
};

// Sizes of every workspace region; the same function both sizes and carves.
long long carve(int n, long long nnz, int t_cap, char* base, GraphDev* g, int flags = 0) {
    Layout L;
    const long long N = n;
    const long long nch = nnz / dsg::MIN_CH + 2;
    const long long ntiles = (N + 4095) / 4096 + 1;
    const long long rtiles = (N + 4095) / 4096 + 1;
    long long o_ctl = L.add(dsg::ctl_bytes());
    long long o_gs = L.add(sizeof(dsg::GridSync));
    long long o_load = L.add(4 * N), o_prio = L.add(4 * N), o_rnd = L.add(4 * N), o_inc = L.add(4 * N);
    long long o_order = L.add(4 * N), o_best = L.add(4 * N);
    long long o_kA = L.add(4 * N), o_kB = L.add(4 * N), o_vA = L.add(4 * N), o_vB = L.add(4 * N);
    long long o_L0 = L.add(4 * N), o_L1 = L.add(4 * N), o_iv = L.add(4 * N), o_ie = L.add(4 * (N + 1));
    long long o_ir = L.add(4 * N), o_sir = L.add(4 * N), o_iv1 = L.add(4 * N), o_st2 = L.add(4 * ((N + 15) / 16 + 1));
    long long o_siv = L.add(4 * N), o_sie = L.add(4 * (N + 1)), o_A = L.add(4 * N);
    long long o_cf = L.add(4 * nch), o_cl = L.add(4 * nch), o_scf = L.add(4 * nch), o_scl = L.add(4 * nch);
    long long o_ts = L.add(8 * ntiles), o_to = L.add(8 * ntiles), o_tb = L.add(24 * ntiles);
    long long o_rh = L.add(4 * 256 * rtiles);
    long long o_he = L.add(8LL * t_cap), o_hv = L.add(8LL * t_cap), o_hi = L.add(4LL * t_cap);
    long long o_rd = L.add(4LL * t_cap), o_dg = L.add(8LL * t_cap), o_hw = L.add(4LL * t_cap), o_hl = L.add(4LL * t_cap);
    int lbits = 0, sbits = 0;
    const bool bucketed = dsg::bucket_params(N, &lbits, &sbits);
    long long o_bkt = L.add(bucketed ? 4 * nnz : 0), o_bf = L.add(4 * dsg::BKT_MAX_NR);
    long long o_rb = L.add(4 * (dsg::BKT_MAX_NR + 1));
    long long o_cb = L.add(4 * ((N + 7) / 8 + 1)), o_crb = L.add(4 * 16), o_crs = L.add(4 * (1 << 17));
    long long o_crt = L.add(8 * ((1 << 17) / 1024));
    long long o_seg = L.add(4 * 6 * dsg::PEEL_BLK);
    long long o_n0 = L.add(4 * N), o_n1 = L.add(4 * N), o_x0 = L.add(4 * N), o_x1 = L.add(4 * N);
    long long o_sf = L.add(4 * 4 * dsg::PEEL_BLK), o_sn = L.add(4 * 4 * dsg::PEEL_BLK);
    if (base && g) {
        g->N0 = reinterpret_cast<int*>(base + o_n0);
        g->N1 = reinterpret_cast<int*>(base + o_n1);
        g->X0 = reinterpret_cast<int*>(base + o_x0);
        g->X1 = reinterpret_cast<int*>(base + o_x1);
        g->segF = reinterpret_cast<int*>(base + o_sf);
        g->segN = reinterpret_cast<int*>(base + o_sn);
        g->cr_samp = reinterpret_cast<int*>(base + o_crs);
        g->cr_tsum = reinterpret_cast<long long*>(base + o_crt);
        g->seg = reinterpret_cast<int*>(base + o_seg);
        g->cb = reinterpret_cast<unsigned int*>(base + o_cb);
        g->cr_bounds = reinterpret_cast<int*>(base + o_crb);
        g->rshift = bucketed ? lbits : 0;
        if (flags & DSG_HUB_ORDER) {
            g->bm = dsg::BktMap{sbits, dsg::BKT_LINE, dsg::BKT_HUB_IDS};
            g->nr = bucketed ? 1 << sbits : 0;
        } else {
            // contiguous ranges of 2^lbits ids; only the first ceil(n / 2^lbits) hold vertices
            g->bm = dsg::BktMap{sbits, lbits, 0};
            g->nr = bucketed ? (int)((N + (1LL << lbits) - 1) >> lbits) : 0;
        }
        g->rbase = reinterpret_cast<int*>(base + o_rb);
        g->bkt = reinterpret_cast<int*>(base + o_bkt);
        g->bfill = reinterpret_cast<unsigned int*>(base + o_bf);
        g->ctl = reinterpret_cast<dsg::Ctl*>(base + o_ctl);
        g->gsync = reinterpret_cast<dsg::GridSync*>(base + o_gs);
        g->load = reinterpret_cast<int*>(base + o_load);
        g->prio = reinterpret_cast<int*>(base + o_prio);
        g->rnd = reinterpret_cast<int*>(base + o_rnd);
        g->inc = reinterpret_cast<int*>(base + o_inc);
        g->order = reinterpret_cast<int*>(base + o_order);
        g->best_order = reinterpret_cast<int*>(base + o_best);
        g->kA = reinterpret_cast<int*>(base + o_kA);
        g->kB = reinterpret_cast<int*>(base + o_kB);
        g->vA = reinterpret_cast<int*>(base + o_vA);
        g->vB = reinterpret_cast<int*>(base + o_vB);
        g->L0 = reinterpret_cast<int*>(base + o_L0);
        g->L1 = reinterpret_cast<int*>(base + o_L1);
        g->iv = reinterpret_cast<int*>(base + o_iv);
        g->ie = reinterpret_cast<int*>(base + o_ie);
        g->siv = reinterpret_cast<int*>(base + o_siv);
        g->sie = reinterpret_cast<int*>(base + o_sie);
        g->A = reinterpret_cast<int*>(base + o_A);
        g->ir = reinterpret_cast<int*>(base + o_ir);
        g->iv1 = reinterpret_cast<int*>(base + o_iv1);
        g->st2 = reinterpret_cast<unsigned int*>(base + o_st2);
        g->sir = reinterpret_cast<int*>(base + o_sir);
        g->cfirst = reinterpret_cast<int*>(base + o_cf);
        g->clast = reinterpret_cast<int*>(base + o_cl);
        g->scf = reinterpret_cast<int*>(base + o_scf);
        g->scl = reinterpret_cast<int*>(base + o_scl);
        g->tile_sum = reinterpret_cast<long long*>(base + o_ts);
        g->tile_off = reinterpret_cast<long long*>(base + o_to);
        g->tile_best = reinterpret_cast<long long*>(base + o_tb);
        g->rhist = reinterpret_cast<int*>(base + o_rh);
        g->hist_e = reinterpret_cast<long long*>(base + o_he);
        g->hist_v = reinterpret_cast<long long*>(base + o_hv);
        g->hist_i = reinterpret_cast<int*>(base + o_hi);
        g->rounds = reinterpret_cast<int*>(base + o_rd);
        g->digest = reinterpret_cast<unsigned long long*>(base + o_dg);
        g->hist_w = reinterpret_cast<int*>(base + o_hw);
        g->hist_lmax = reinterpret_cast<int*>(base + o_hl);
    }
    if (flags & DSG_HUB_ORDER) {
        // the renumbered CSR and the two permutations; graph_init fills them
        // and points off / adj / perm / iperm there
        const long long o_hoff = L.add(4 * (N + 1)), o_hadj = L.add(4 * nnz);
        const long long o_perm = L.add(4 * N), o_iperm = L.add(4 * N);
        if (base && g) {
            g->hub_off = reinterpret_cast<int*>(base + o_hoff);
            g->hub_adj = reinterpret_cast<int*>(base + o_hadj);
            g->hub_perm = reinterpret_cast<int*>(base + o_perm);
            g->hub_iperm = reinterpret_cast<int*>(base + o_iperm);
        }
    }
    return L.total;
}

const char* err_name(int code) {
    switch (code) {
        case dsg::ERR_OFF_FIRST: return "offsets[0] != 0";
        case dsg::ERR_OFF_LAST: return "offsets[n] != nnz";
        case dsg::ERR_OFF_DECREASING: return "offsets decrease";
        case dsg::ERR_ADJ_RANGE: return "adjacency entry outside [0, n)";
        case dsg::ERR_SELF_LOOP: return "self-loop";
        case dsg::ERR_ROW_ORDER: return "row not strictly increasing (unsorted or duplicate entry)";
        case dsg::ERR_ASYMMETRIC: return "CSR not symmetric";
        case dsg::ERR_INTERNAL: return "internal consistency check failed";
        default: return "unknown";
    }
}

dsg_status read_ctl(dsg_graph* g, dsg::Ctl* out) {
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    DSG_HIP(hipMemcpy(out, g->d.ctl, sizeof(dsg::Ctl), hipMemcpyDeviceToHost), "hipMemcpy(ctl)");
    return DSG_OK;
}

dsg_status check_errors(dsg_graph* g, const char* stage) {
    dsg::Ctl c;
    dsg_status st = read_ctl(g, &c);
    if (st != DSG_OK) return st;
    if (c.err_count != 0) {
        char buf[256];
        snprintf(buf, sizeof buf, "invalid CSR (%s): %s at %s %d (%d problems)", stage, err_name(c.err_code),
                 c.err_code == dsg::ERR_ADJ_RANGE ? "entry" : "vertex", c.err_vertex, c.err_count);
        return fail(DSG_EINVAL, buf);
    }
    return DSG_OK;
}

}  // namespace

extern "C" {

const char* dsg_last_error(void) { return g_err.c_str(); }

dsg_status dsg_ctx_create(int device, void* hip_stream, dsg_ctx** out) {
    if (!out) return fail(DSG_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    DSG_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(DSG_EDEVICE, "no such device");
    DSG_HIP(hipSetDevice(device), "hipSetDevice");
    resolve_scratch(device);  // a failure is reported by dsg_par_run_noalloc only
    hipDeviceProp_t prop;
    DSG_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (!prop.cooperativeLaunch) return fail(DSG_EDEVICE, "device lacks cooperative launch");
    dsg_ctx* c = new (std::nothrow) dsg_ctx();
    if (!c) return fail(DSG_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->num_cu = prop.multiProcessorCount;
    int per_cu = dsg::peel_blocks_per_cu();
    // one block per CU: the round loop's grid syncs cost more with more
    // blocks, and 1024 threads per CU keep enough loads in flight
    if (per_cu < 1) return fail(DSG_EDEVICE, "round kernel cannot be resident");
    c->peel_grid = c->num_cu * (per_cu < dsg::PEEL_BLOCKS_PER_CU ? per_cu : dsg::PEEL_BLOCKS_PER_CU);
    c->sort_grid = c->num_cu * 8;
    *out = c;
    return DSG_OK;
}

dsg_status dsg_ctx_destroy(dsg_ctx* ctx) {
    delete ctx;
    return DSG_OK;
}

dsg_status dsg_workspace_bytes(int32_t n, int64_t nnz, int32_t t_cap, int64_t* bytes) {
    if (!bytes) return fail(DSG_EINVAL, "bytes is NULL");
    if (n < 1) return fail(DSG_EINVAL, "n must be >= 1");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    if (t_cap < 1) return fail(DSG_EINVAL, "t_cap must be >= 1");
    *bytes = carve(n, nnz, t_cap, nullptr, nullptr);
    return DSG_OK;
}

dsg_status dsg_workspace_bytes_ex(int32_t n, int64_t nnz, int32_t t_cap, int32_t flags, int64_t* bytes) {
    const dsg_status st = dsg_workspace_bytes(n, nnz, t_cap, bytes);
    if (st != DSG_OK) return st;
    *bytes = carve(n, nnz, t_cap, nullptr, nullptr, flags);
    return DSG_OK;
}

}  // extern "C"

namespace {

// Binds a device CSR to caller storage *g (value-initialised): carves the
// workspace, checks the CSR, builds the static items and resets the state.
// `events`: create the two events that time each dsg_run.  Graphs made inside
// the library (Pruning-and-Refining) skip them, so those calls create no HIP
// objects.  On failure *g holds nothing to release.
dsg_status graph_init(dsg_graph* g, dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets,
                      const int32_t* d_adj, void* d_workspace, int64_t workspace_bytes, int32_t t_cap, int32_t flags,
                      bool events) {
    if (!ctx || !d_offsets || !d_workspace) return fail(DSG_EINVAL, "NULL argument");
    if (n < 1) return fail(DSG_EINVAL, "n must be >= 1");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    if (nnz > 0 && !d_adj) return fail(DSG_EINVAL, "adj is NULL");
    if (t_cap < 1) return fail(DSG_EINVAL, "t_cap must be >= 1");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(DSG_EINVAL, "workspace not 256-byte aligned");
    if (flags & ~(DSG_VALIDATE | DSG_HUB_ORDER)) return fail(DSG_EINVAL, "unknown flags");
    long long need = carve(n, nnz, t_cap, nullptr, nullptr, flags);
    if (workspace_bytes < need) return fail(DSG_ENOMEM, "workspace smaller than dsg_workspace_bytes_ex()");
    DSG_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    g->ctx = ctx;
    g->ws = static_cast<char*>(d_workspace);
    g->ws_bytes = workspace_bytes;
    g->t_cap = t_cap;
    g->last_variant = -1;
    g->bkt_min_e = (flags & DSG_HUB_ORDER) ? dsg::BKT_HUB_DEFAULT_MIN_E : dsg::BKT_DEFAULT_MIN_E;
    g->coarse_min_e = -1;
    g->sort_coarse = -1;
    g->peel_select = -1;
    g->d.n = n;
    g->d.nnz = nnz;
    g->d.off = d_offsets;
    g->d.adj = d_adj;
    carve(n, nnz, t_cap, g->ws, &g->d, flags);
    hipStream_t s = ctx->stream;
    hipError_t e;
    if ((e = dsg::launch_zero_ctl(g->d, s)) != hipSuccess) return hip_fail(e, "zero ctl");
    if ((e = dsg::launch_check_offsets(g->d, s)) != hipSuccess) return hip_fail(e, "check offsets");
    dsg_status st = check_errors(g, "offsets");
    if (st != DSG_OK) return st;
    if ((e = dsg::launch_check_range(g->d, s)) != hipSuccess) return hip_fail(e, "check range");
    st = check_errors(g, "entries");
    if (st != DSG_OK) return st;
    // offsets and entries are in range now, so the static item list (which
    // the row check walks) can be built
    if ((e = dsg::launch_build_static_items(g->d, s)) != hipSuccess) return hip_fail(e, "static items");
    dsg::Ctl c;
    st = read_ctl(g, &c);
    if (st != DSG_OK) return st;
    g->d.max_deg = c.max_deg;
    if (flags & DSG_VALIDATE) {
        if ((e = dsg::launch_check_rows(g->d, s)) != hipSuccess) return hip_fail(e, "check rows");
        st = check_errors(g, "rows");
        if (st != DSG_OK) return st;
    }
    if (flags & DSG_HUB_ORDER) {
        // renumber into the workspace, then work on the renumbered CSR only
        if ((e = dsg::launch_hub_order(g->d, c.max_deg, g->d.hub_off, g->d.hub_adj, g->d.hub_perm, g->d.hub_iperm,
                                       s)) != hipSuccess)
            return hip_fail(e, "hub order");
        g->d.off = g->d.hub_off;
        g->d.adj = g->d.hub_adj;
        g->d.perm = g->d.hub_perm;
        g->d.iperm = g->d.hub_iperm;
        if ((e = dsg::launch_build_static_items(g->d, s)) != hipSuccess) return hip_fail(e, "static items");
    }
    long long items = 0;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = hipMemcpy(&items, g->d.tile_off, sizeof(long long), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(items)");
    g->d.n_items = (int)items;
    if ((flags & DSG_HUB_ORDER) && g->d.nr > 0 && n > dsg::BKT_HUB_IDS) {
        // narrow bucket apply: ranges of 2^16 local ids, when every vertex past
        // the hub ids (internal ids by non-increasing degree) has degree < 2^16
        int cl = 0;
        while ((1LL << cl) < (long long)n) cl++;
        const int sb = cl - dsg::BKT_NARROW_SHIFT;
        int od[2] = {0, 0};
        if (sb >= dsg::BKT_NARROW_MIN_SB && (1 << sb) <= dsg::BKT_MAX_NR) {
            if ((e = hipMemcpy(od, g->d.hub_off + dsg::BKT_HUB_IDS, sizeof od, hipMemcpyDeviceToHost)) != hipSuccess)
                return hip_fail(e, "hipMemcpy(degree)");
            if (od[1] - od[0] < (1 << 16)) {
                g->d.narrow = 1;
                g->d.rshift = dsg::BKT_NARROW_SHIFT;
                g->d.bm = dsg::BktMap{sb, dsg::BKT_LINE, dsg::BKT_HUB_IDS};
                g->d.nr = 1 << sb;
            }
        }
    }
    if ((e = dsg::launch_bucket_bases(g->d, s)) != hipSuccess) return hip_fail(e, "bucket bases");
    if ((e = dsg::launch_reset_state(g->d, s)) != hipSuccess) return hip_fail(e, "reset");
    if (events) {
        if ((e = hipEventCreate(&g->ev0)) != hipSuccess) {
            g->ev0 = nullptr;
            return hip_fail(e, "hipEventCreate");
        }
        if ((e = hipEventCreate(&g->ev1)) != hipSuccess) {
            (void)hipEventDestroy(g->ev0);
            g->ev0 = g->ev1 = nullptr;
            return hip_fail(e, "hipEventCreate");
        }
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        if (g->ev0) (void)hipEventDestroy(g->ev0);
        if (g->ev1) (void)hipEventDestroy(g->ev1);
        g->ev0 = g->ev1 = nullptr;
        return hip_fail(e, "hipStreamSynchronize");
    }
    return DSG_OK;
}

// Releases the HIP objects a graph holds (not its storage or workspace).
void graph_fini(dsg_graph* g) {
    for (hipEvent_t ev : g->kev) (void)hipEventDestroy(ev);
    g->kev.clear();
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    g->ev0 = g->ev1 = nullptr;
    if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->gexec = nullptr;
    g->cap_stream = nullptr;
}

}  // namespace

extern "C" {

dsg_status dsg_graph_create(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                            void* d_workspace, int64_t workspace_bytes, int32_t t_cap, int32_t flags,
                            dsg_graph** out) {
    if (!out) return fail(DSG_EINVAL, "NULL argument");
    *out = nullptr;
    dsg_graph* g = new (std::nothrow) dsg_graph();
    if (!g) return fail(DSG_ENOMEM, "host allocation failed");
    const dsg_status st = graph_init(g, ctx, n, nnz, d_offsets, d_adj, d_workspace, workspace_bytes, t_cap, flags,
                                     true);
    if (st != DSG_OK) {
        delete g;
        return st;
    }
    *out = g;
    return DSG_OK;
}

dsg_status dsg_run(dsg_graph* g, int32_t T, int32_t eps_num, int32_t eps_den, dsg_variant variant) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    if (T < 0) return fail(DSG_EINVAL, "T must be >= 0");
    if (eps_num < 0 || eps_den < 1) return fail(DSG_EINVAL, "eps must be eps_num >= 0, eps_den >= 1");
    if (variant != DSG_SEQ && variant != DSG_PEEL && variant != DSG_SORT && variant != DSG_PEEL_MONO)
        return fail(DSG_EINVAL, "unknown variant");
    if ((long long)g->recorded + T > g->t_cap) return fail(DSG_EINVAL, "T exceeds the history capacity t_cap");
    if (variant == DSG_SEQ && g->d.n > dsg::SEQ_MAX_N) return fail(DSG_EINVAL, "DSG_SEQ supports n <= 16000");
    if ((variant == DSG_PEEL || variant == DSG_PEEL_MONO) && g->d.n >= dsg::PEEL_MAX_N)
        return fail(DSG_EINVAL, "DSG_PEEL and DSG_PEEL_MONO support n < 2^26");
    // loads grow by at most max_degree per iteration; priorities add one more
    if (g->load_bound + ((long long)T + 1) * (long long)g->d.max_deg >= (1LL << 31))
        return fail(DSG_EOVERFLOW, "loads could exceed 31 bits");
    DSG_HIP(hipSetDevice(g->ctx->device), "hipSetDevice");
    hipStream_t s = g->ctx->stream;
    if (g->ktime) {
        while ((int)g->kev.size() < 2 * T) {
            hipEvent_t ev;
            DSG_HIP(hipEventCreate(&ev), "hipEventCreate");
            g->kev.push_back(ev);
        }
    }
    g->klaunches = 0;
    // every launch of the T iterations, on stream `qs` (`timed`: events around
    // each iteration's dominant kernel)
    auto enqueue_run = [&](hipStream_t qs, bool timed) -> hipError_t {
        for (int t = 0; t < T; t++) {
            const int slot = g->recorded + t;
            hipEvent_t ea = timed ? g->kev[2 * t] : nullptr;
            hipEvent_t eb = timed ? g->kev[2 * t + 1] : nullptr;
            hipError_t e;
            if (variant == DSG_PEEL || variant == DSG_PEEL_MONO) {
                const bool near = g->peel_select > 0 ||
                                  (g->peel_select < 0 && dsg::NEAR_DEFAULT_MIN_N > 0 && g->d.n >= dsg::NEAR_DEFAULT_MIN_N);
                e = dsg::enqueue_iter_peel(g->d, slot, eps_num, eps_den, g->ctx->peel_grid, g->bkt_min_e,
                                           g->coarse_min_e >= 0 ? g->coarse_min_e : dsg::PEEL_DEFAULT_COARSE_MIN_E,
                                           variant == DSG_PEEL_MONO, near, qs, ea, eb);
            } else if (variant == DSG_SORT) {
                long long bound = g->load_bound + (long long)t * (long long)g->d.max_deg;
                int bits = 0;
                while (bits < 31 && (bound >> bits) != 0) bits++;
                const bool coarse =
                    g->sort_coarse > 0 ||
                    (g->sort_coarse < 0 && g->d.n >= dsg::SORT_COARSE_MIN_N && g->d.n <= dsg::SORT_COARSE_MAX_N);
                e = dsg::enqueue_iter_sort(g->d, slot, bits, g->ctx->sort_grid, coarse && g->d.n < (1 << 26), qs,
                                           ea, eb);
            } else {
                e = dsg::enqueue_iter_seq(g->d, slot, qs, ea, eb);
            }
            if (e != hipSuccess) return e;
            if (timed) g->klaunches++;
        }
        return hipSuccess;
    };
    if (g->ev0) DSG_HIP(hipEventRecord(g->ev0, s), "hipEventRecord");
    bool launched = false;
    if (g->replay && !g->ktime && g->replay_state >= 0 && T > 0) {
        // everything the launches depend on besides the device state
        const long long key[11] = {T, eps_num, eps_den, (long long)variant, g->recorded, g->load_bound,
                                   g->bkt_min_e, g->coarse_min_e, g->sort_coarse,
                                   (long long)reinterpret_cast<uintptr_t>(g->d.rmin), g->peel_select};
        if (!(g->gexec && memcmp(key, g->gkey, sizeof key) == 0)) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t ex = nullptr;
            hipError_t e = g->cap_stream ? hipSuccess : hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t eq = enqueue_run(g->cap_stream, false);
                e = hipStreamEndCapture(g->cap_stream, &graph);  // always ends the capture
                if (eq != hipSuccess) e = eq;
            }
            if (e == hipSuccess && graph) e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e == hipSuccess && ex) {
                if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
                g->gexec = ex;
                memcpy(g->gkey, key, sizeof key);
                g->replay_state = 1;
            } else {
                // the runtime refused to capture some launch: run eagerly
                (void)hipGetLastError();
                if (ex) (void)hipGraphExecDestroy(ex);
                g->replay_state = -1;
            }
        }
        if (g->replay_state == 1) {
            DSG_HIP(hipGraphLaunch(g->gexec, s), "hipGraphLaunch");
            launched = true;
        }
    }
    if (!launched) {
        const hipError_t e = enqueue_run(s, g->ktime);
        if (e != hipSuccess) return hip_fail(e, "enqueue iteration");
    }
    if (g->ev1) DSG_HIP(hipEventRecord(g->ev1, s), "hipEventRecord");
    g->timed = g->ev1 != nullptr;
    g->recorded += T;
    g->iters_done += T;
    g->load_bound += (long long)T * (long long)g->d.max_deg;
    if (T > 0) g->last_variant = variant;
    return DSG_OK;
}

dsg_status dsg_run_until(dsg_graph* g, int32_t T_max, int32_t eps_num, int32_t eps_den, dsg_variant variant,
                         int32_t tol_num, int32_t tol_den, int32_t* iters, int32_t* certified) {
    if (!g || !iters || !certified) return fail(DSG_EINVAL, "NULL argument");
    if (T_max < 0) return fail(DSG_EINVAL, "T_max must be >= 0");
    if (tol_num < 0 || tol_den < 1) return fail(DSG_EINVAL, "tolerance must be tol_num >= 0, tol_den >= 1");
    *iters = 0;
    *certified = 0;
    for (int t = 0; t < T_max; t++) {
        dsg_status st = dsg_run(g, 1, eps_num, eps_den, variant);
        if (st != DSG_OK) return st;
        *iters = t + 1;
        dsg::Ctl c;
        st = read_ctl(g, &c);
        if (st != DSG_OK) return st;
        if (c.err_count != 0) return fail(DSG_EDEVICE, "a kernel consistency check failed");
        int lmax = 0;
        DSG_HIP(hipMemcpy(&lmax, g->d.hist_lmax + (g->recorded - 1), sizeof(int), hipMemcpyDeviceToHost),
                "hipMemcpy(largest load)");
        // rho* <= L_t / t, so L_t * v * den <= t * e * (den + num) certifies rho(best) >= rho* / (1 + tol)
        const __int128 lhs = (__int128)lmax * c.best_v * tol_den;
        const __int128 rhs = (__int128)g->iters_done * c.best_e * ((__int128)tol_den + tol_num);
        if (lhs <= rhs) {
            *certified = 1;
            break;
        }
    }
    return DSG_OK;
}

dsg_status dsg_reset(dsg_graph* g) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    DSG_HIP(hipSetDevice(g->ctx->device), "hipSetDevice");
    hipError_t e = dsg::launch_reset_state(g->d, g->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "reset");
    g->recorded = 0;
    g->iters_done = 0;
    g->load_bound = 0;
    g->last_variant = -1;
    g->timed = false;
    return DSG_OK;
}

dsg_status dsg_sync(dsg_graph* g) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    dsg::Ctl c;
    dsg_status st = read_ctl(g, &c);
    if (st != DSG_OK) return st;
    if (c.err_count != 0) return fail(DSG_EDEVICE, "a kernel consistency check failed");
    return DSG_OK;
}

dsg_status dsg_last_run_ms(dsg_graph* g, float* ms) {
    if (!g || !ms) return fail(DSG_EINVAL, "NULL argument");
    if (!g->timed) return fail(DSG_ESTATE, "no run recorded");
    DSG_HIP(hipEventSynchronize(g->ev1), "hipEventSynchronize");
    DSG_HIP(hipEventElapsedTime(ms, g->ev0, g->ev1), "hipEventElapsedTime");
    return DSG_OK;
}

dsg_status dsg_set_peel_tuning(dsg_graph* g, int64_t bucket_min_edges, int64_t coarse_min_edges) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    if (bucket_min_edges < -1 || coarse_min_edges < -1) return fail(DSG_EINVAL, "thresholds must be >= -1");
    g->bkt_min_e = bucket_min_edges >= 0 ? bucket_min_edges
                   : g->d.perm              ? dsg::BKT_HUB_DEFAULT_MIN_E
                                            : dsg::BKT_DEFAULT_MIN_E;
    g->coarse_min_e = coarse_min_edges;
    return DSG_OK;
}

dsg_status dsg_set_sort_tuning(dsg_graph* g, int32_t coarse_ranks) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    if (coarse_ranks < -1 || coarse_ranks > 1) return fail(DSG_EINVAL, "coarse_ranks must be -1, 0 or 1");
    g->sort_coarse = coarse_ranks;
    return DSG_OK;
}

dsg_status dsg_set_peel_select(dsg_graph* g, int32_t mode) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    if (mode < -1 || mode > 1) return fail(DSG_EINVAL, "mode must be -1, 0 or 1");
    g->peel_select = mode;
    return DSG_OK;
}

dsg_status dsg_set_graph_replay(dsg_graph* g, int32_t enable) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    g->replay = enable != 0;
    if (g->replay && g->replay_state < 0) g->replay_state = 0;  // allow another capture attempt
    return DSG_OK;
}

dsg_status dsg_get_graph_replay(dsg_graph* g, int32_t* state) {
    if (!g || !state) return fail(DSG_EINVAL, "NULL argument");
    *state = g->replay ? g->replay_state : 0;
    return DSG_OK;
}

dsg_status dsg_set_kernel_timing(dsg_graph* g, int32_t enable) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    g->ktime = enable != 0;
    return DSG_OK;
}

dsg_status dsg_get_kernel_timing(dsg_graph* g, float* total_ms, int32_t* launches) {
    if (!g || !total_ms || !launches) return fail(DSG_EINVAL, "NULL argument");
    float tot = 0.f;
    for (int i = 0; i < g->klaunches; i++) {
        float ms = 0.f;
        DSG_HIP(hipEventSynchronize(g->kev[2 * i + 1]), "hipEventSynchronize");
        DSG_HIP(hipEventElapsedTime(&ms, g->kev[2 * i], g->kev[2 * i + 1]), "hipEventElapsedTime");
        tot += ms;
    }
    *total_ms = tot;
    *launches = g->klaunches;
    return DSG_OK;
}

dsg_status dsg_get_best(dsg_graph* g, int64_t* edges, int64_t* verts, int32_t* iter, int32_t* index) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    dsg::Ctl c;
    dsg_status st = read_ctl(g, &c);
    if (st != DSG_OK) return st;
    if (edges) *edges = c.best_e;
    if (verts) *verts = c.best_v;
    if (iter) *iter = c.best_iter;
    if (index) *index = (int32_t)c.best_idx;
    return DSG_OK;
}

// Under hub order: the caller's id of every internal vertex (empty otherwise).
static dsg_status read_perm(dsg_graph* g, std::vector<int32_t>* perm) {
    perm->clear();
    if (!g->d.perm) return DSG_OK;
    perm->resize((size_t)g->d.n);
    DSG_HIP(hipMemcpy(perm->data(), g->d.perm, sizeof(int32_t) * (size_t)g->d.n, hipMemcpyDeviceToHost),
            "hipMemcpy(perm)");
    return DSG_OK;
}

dsg_status dsg_get_best_mask(dsg_graph* g, uint8_t* h_mask) {
    if (!g || !h_mask) return fail(DSG_EINVAL, "NULL argument");
    dsg::Ctl c;
    dsg_status st = read_ctl(g, &c);
    if (st != DSG_OK) return st;
    const int n = g->d.n;
    if (c.best_iter == 0) {
        memset(h_mask, 1, (size_t)n);
        return DSG_OK;
    }
    std::vector<int32_t> ord((size_t)n);
    DSG_HIP(hipMemcpy(ord.data(), g->d.best_order, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost),
            "hipMemcpy(best order)");
    std::vector<int32_t> perm;
    if ((st = read_perm(g, &perm)) != DSG_OK) return st;
    memset(h_mask, 0, (size_t)n);
    for (long long i = c.best_idx; i < n; i++) {
        const int v = ord[(size_t)i];
        h_mask[perm.empty() ? v : perm[(size_t)v]] = 1;
    }
    return DSG_OK;
}

dsg_status dsg_get_loads(dsg_graph* g, int64_t* h_loads) {
    if (!g || !h_loads) return fail(DSG_EINVAL, "NULL argument");
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    std::vector<int32_t> tmp((size_t)g->d.n), perm;
    DSG_HIP(hipMemcpy(tmp.data(), g->d.load, sizeof(int32_t) * (size_t)g->d.n, hipMemcpyDeviceToHost),
            "hipMemcpy(loads)");
    const dsg_status st = read_perm(g, &perm);
    if (st != DSG_OK) return st;
    for (int v = 0; v < g->d.n; v++) h_loads[perm.empty() ? v : perm[(size_t)v]] = tmp[(size_t)v];
    return DSG_OK;
}

dsg_status dsg_get_iter_densities(dsg_graph* g, int64_t* h_edges, int64_t* h_verts, int32_t* h_index, int32_t cap,
                                  int32_t* count) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    const int k = cap < g->recorded ? cap : g->recorded;
    if (k > 0) {
        if (h_edges)
            DSG_HIP(hipMemcpy(h_edges, g->d.hist_e, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        if (h_verts)
            DSG_HIP(hipMemcpy(h_verts, g->d.hist_v, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        if (h_index)
            DSG_HIP(hipMemcpy(h_index, g->d.hist_i, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
    }
    if (count) *count = g->recorded;
    return DSG_OK;
}

dsg_status dsg_get_order(dsg_graph* g, int32_t* h_round, int32_t* h_pos, int32_t* n_rounds) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    if (g->last_variant < 0) return fail(DSG_ESTATE, "no iteration has run");
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    const int n = g->d.n;
    std::vector<int32_t> perm;
    const dsg_status st = read_perm(g, &perm);
    if (st != DSG_OK) return st;
    if (h_round) {
        if (perm.empty()) {
            DSG_HIP(hipMemcpy(h_round, g->d.rnd, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost),
                    "hipMemcpy(round)");
        } else {
            std::vector<int32_t> rnd((size_t)n);
            DSG_HIP(hipMemcpy(rnd.data(), g->d.rnd, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost),
                    "hipMemcpy(round)");
            for (int v = 0; v < n; v++) h_round[perm[(size_t)v]] = rnd[(size_t)v];
        }
    }
    if (h_pos) {
        std::vector<int32_t> ord((size_t)n);
        DSG_HIP(hipMemcpy(ord.data(), g->d.order, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost),
                "hipMemcpy(order)");
        for (int i = 0; i < n; i++) {
            const int v = ord[(size_t)i];
            h_pos[perm.empty() ? v : perm[(size_t)v]] = i;
        }
    }
    if (n_rounds) {
        int r = 0;
        DSG_HIP(hipMemcpy(&r, g->d.rounds + (g->recorded - 1), sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy(rounds)");
        *n_rounds = r;
    }
    return DSG_OK;
}

dsg_status dsg_get_iter_bounds(dsg_graph* g, int32_t* h_width, int64_t* h_load_max, int32_t cap, int32_t* count) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    const int k = cap < g->recorded ? cap : g->recorded;
    if (k > 0) {
        std::vector<int32_t> tmp((size_t)k);
        if (h_width)
            DSG_HIP(hipMemcpy(h_width, g->d.hist_w, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(width)");
        if (h_load_max) {
            DSG_HIP(hipMemcpy(tmp.data(), g->d.hist_lmax, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(lmax)");
            for (int i = 0; i < k; i++) h_load_max[i] = tmp[(size_t)i];
        }
    }
    if (count) *count = g->recorded;
    return DSG_OK;
}

dsg_status dsg_get_iter_digests(dsg_graph* g, uint64_t* h_digest, int32_t* h_rounds, int32_t cap, int32_t* count) {
    if (!g) return fail(DSG_EINVAL, "graph is NULL");
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    const int k = cap < g->recorded ? cap : g->recorded;
    if (k > 0) {
        if (h_digest)
            DSG_HIP(hipMemcpy(h_digest, g->d.digest, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(digest)");
        if (h_rounds)
            DSG_HIP(hipMemcpy(h_rounds, g->d.rounds, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(rounds)");
    }
    if (count) *count = g->recorded;
    return DSG_OK;
}

dsg_status dsg_graph_destroy(dsg_graph* g) {
    if (!g) return DSG_OK;
    graph_fini(g);
    delete g;
    return DSG_OK;
}

// ------------------------------------------------ Pruning-and-Refining

}  // extern "C"

namespace {

struct ParWs {
    char* gws;
    long long gws_bytes;
    int* core;
    int* rv;
    int* kmax;
    int* apx;    // approximate core numbers, input ids
    int* core1;  // exact core numbers of the approximate cut, its own ids
    int* off[2];
    int* adj[2];
    int* oldid[2];
    int* iota;
    int* load;
    int* keep;
    int* newid;
    int* f;
    int* fs;
    long long* tiles;
    long long* counts;
    unsigned char* mask;
};

long long carve_par(int n, long long nnz, int T, char* base, ParWs* w) {
    Layout L;
    const long long N = n, E = nnz;
    const long long gb = carve(n, nnz, T, nullptr, nullptr);
    long long o_g = L.add(gb);
    long long o_core = L.add(4 * N), o_rv = L.add(4 * (N + 1)), o_km = L.add(16);
    long long o_apx = L.add(4 * N), o_core1 = L.add(4 * N);
    long long o_off0 = L.add(4 * (N + 1)), o_adj0 = L.add(4 * (E > 0 ? E : 1));
    long long o_off1 = L.add(4 * (N + 1)), o_adj1 = L.add(4 * (E > 0 ? E : 1));
    long long o_id0 = L.add(4 * N), o_id1 = L.add(4 * N), o_iota = L.add(4 * N), o_load = L.add(4 * N);
    long long o_keep = L.add(4 * (N + 1)), o_newid = L.add(4 * (N + 1));
    long long o_f = L.add(4 * (E + 1)), o_fs = L.add(4 * (E + 1));
    long long o_t = L.add(8 * dsg::par_scan_tiles((N > E ? N : E) + 1)), o_c = L.add(16), o_m = L.add(N);
    if (base && w) {
        w->gws = base + o_g;
        w->gws_bytes = gb;
        w->core = reinterpret_cast<int*>(base + o_core);
        w->rv = reinterpret_cast<int*>(base + o_rv);
        w->kmax = reinterpret_cast<int*>(base + o_km);
        w->apx = reinterpret_cast<int*>(base + o_apx);
        w->core1 = reinterpret_cast<int*>(base + o_core1);
        w->off[0] = reinterpret_cast<int*>(base + o_off0);
        w->adj[0] = reinterpret_cast<int*>(base + o_adj0);
        w->off[1] = reinterpret_cast<int*>(base + o_off1);
        w->adj[1] = reinterpret_cast<int*>(base + o_adj1);
        w->oldid[0] = reinterpret_cast<int*>(base + o_id0);
        w->oldid[1] = reinterpret_cast<int*>(base + o_id1);
        w->iota = reinterpret_cast<int*>(base + o_iota);
        w->load = reinterpret_cast<int*>(base + o_load);
        w->keep = reinterpret_cast<int*>(base + o_keep);
        w->newid = reinterpret_cast<int*>(base + o_newid);
        w->f = reinterpret_cast<int*>(base + o_f);
        w->fs = reinterpret_cast<int*>(base + o_fs);
        w->tiles = reinterpret_cast<long long*>(base + o_t);
        w->counts = reinterpret_cast<long long*>(base + o_c);
        w->mask = reinterpret_cast<unsigned char*>(base + o_m);
    }
    return L.total;
}

// Cut {x : core[oldid[x]] >= level} out of graph g into CSR buffer `dst`;
// returns the new sizes.  Loads of the kept vertices go to w.load.
dsg_status par_cut(dsg_graph* g, const ParWs& w, const int* core, const int* oldid, int level, int dst, int* n_out,
                   long long* nnz_out) {
    dsg::CoreCut c{oldid, core, level, w.keep, w.newid, w.f, w.fs, w.tiles,
                   w.off[dst], w.adj[dst], w.oldid[dst], w.load, w.counts};
    hipError_t e = dsg::launch_get_core(g->d, c, g->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "getCore");
    long long cnt[2];
    DSG_HIP(hipStreamSynchronize(g->ctx->stream), "hipStreamSynchronize");
    DSG_HIP(hipMemcpy(cnt, w.counts, sizeof(cnt), hipMemcpyDeviceToHost), "hipMemcpy(core sizes)");
    *n_out = (int)cnt[0];
    *nnz_out = cnt[1];
    return DSG_OK;
}

// Core numbers of a CSR into core_out / w.kmax: one DSG_PEEL_MONO pass with
// zero loads and eps = eps_num / eps_den: exact with eps = 0, otherwise the
// (1 + eps)-approximate decomposition (core <= khat <= (1 + eps) core).
// Leaves the graph alive in *gout (its static items serve the next cut).
dsg_status par_coreness(dsg_ctx* ctx, const ParWs& w, int n, long long nnz, const int32_t* d_offsets,
                        const int32_t* d_adj, int tcap, int flags, bool timed, int eps_num, int eps_den, int* core_out,
                        dsg_graph* gb, dsg_graph** gout, int* nrounds_out, int* kmax_out, float* ms_out) {
    *gb = dsg_graph();
    // the framework's graphs keep the input ids (its workspace has no room for a renumbered copy)
    dsg_status st = graph_init(gb, ctx, n, nnz, d_offsets, d_adj, w.gws, w.gws_bytes, tcap, flags & DSG_VALIDATE,
                               false);
    if (st != DSG_OK) return st;
    dsg_graph* g = gb;
    hipStream_t s = ctx->stream;
    if (timed) dsg_set_kernel_timing(g, 1);
    g->d.rmin = w.rv;  // the round loop records each round's minimum (at most n rounds)
    st = dsg_run(g, 1, eps_num, eps_den, DSG_PEEL_MONO);
    g->d.rmin = nullptr;
    if (st != DSG_OK) {
        graph_fini(g);
        return st;
    }
    int nrounds = 0, kmax = 0;
    if (timed) {
        int launches = 0;
        float ms = 0.f;
        dsg_get_kernel_timing(g, &ms, &launches);
        if (ms_out) *ms_out = ms;
        dsg_set_kernel_timing(g, 0);
    }
    hipError_t e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess ||
        (e = hipMemcpy(&nrounds, g->d.rounds, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = dsg::launch_core_numbers(g->d, nrounds, w.rv, core_out, w.kmax, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess ||
        (e = hipMemcpy(&kmax, w.kmax, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) {
        graph_fini(g);
        return hip_fail(e, "core numbers");
    }
    *gout = g;
    *nrounds_out = nrounds;
    *kmax_out = kmax;
    return DSG_OK;
}

}  // namespace

extern "C" {

dsg_status dsg_coreness(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                        void* d_workspace, int64_t workspace_bytes, int32_t flags, int32_t* h_core, int32_t* kmax,
                        int32_t* rounds, float* round_loop_ms) {
    if (!ctx || !d_offsets || !d_workspace || !kmax) return fail(DSG_EINVAL, "NULL argument");
    if (nnz > 0 && !d_adj) return fail(DSG_EINVAL, "d_adj is NULL");
    if (n < 1 || n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "n must be in [1, 2^26)");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    const long long need = carve_par(n, nnz, 1, nullptr, nullptr);
    if (workspace_bytes < need) return fail(DSG_EINVAL, "workspace too small (dsg_par_workspace_bytes with T = 1)");
    DSG_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ParWs w;
    carve_par(n, nnz, 1, static_cast<char*>(d_workspace), &w);
    dsg_graph gb{};
    dsg_graph* g = nullptr;
    int nr = 0, km = 0;
    float ms = 0.f;
    dsg_status st = par_coreness(ctx, w, n, nnz, d_offsets, d_adj, 1, flags, round_loop_ms != nullptr, 0, 1, w.core,
                                 &gb, &g, &nr, &km, &ms);
    if (st != DSG_OK) return st;
    graph_fini(g);
    *kmax = km;
    if (rounds) *rounds = nr;
    if (round_loop_ms) *round_loop_ms = ms;
    if (h_core) DSG_HIP(hipMemcpy(h_core, w.core, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy(core)");
    return DSG_OK;
}

dsg_status dsg_par_workspace_bytes(int32_t n, int64_t nnz, int32_t T, int64_t* bytes) {
    if (!bytes) return fail(DSG_EINVAL, "bytes is NULL");
    if (n < 1 || n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "n must be in [1, 2^26)");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    if (T < 0) return fail(DSG_EINVAL, "T must be >= 0");
    *bytes = carve_par(n, nnz, T > 0 ? T : 1, nullptr, nullptr);
    return DSG_OK;
}

}  // extern "C"

namespace {

// Algorithm 1 with exact (prune 0), approximate (1) or approximate-then-exact
// (2) pruning; see dsg_par_run and dsg_par_run_apx.
dsg_status par_run_impl(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                        void* d_workspace, int64_t workspace_bytes, int32_t T, int32_t eps_num, int32_t eps_den,
                        dsg_variant variant, int32_t flags, int prune, int c_num, int c_den, dsg_par_result* result,
                        dsg_par_apx* apx_out, int64_t* h_iter_edges, int64_t* h_iter_verts, int32_t* h_iter_index,
                        int32_t* h_iter_n, int64_t* h_iter_nnz, int32_t* h_iter_level, uint8_t* h_best_mask,
                        int32_t* h_core, int32_t* h_apx_core) {
    if (!ctx || !d_offsets || !d_workspace || !result) return fail(DSG_EINVAL, "NULL argument");
    if (nnz > 0 && !d_adj) return fail(DSG_EINVAL, "d_adj is NULL");
    if (n < 1 || n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "n must be in [1, 2^26)");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    if (T < 0) return fail(DSG_EINVAL, "T must be >= 0");
    if (eps_num < 0 || eps_den < 1) return fail(DSG_EINVAL, "eps must be eps_num >= 0, eps_den >= 1");
    if (variant != DSG_SEQ && variant != DSG_PEEL && variant != DSG_SORT && variant != DSG_PEEL_MONO)
        return fail(DSG_EINVAL, "unknown variant");
    if (prune != 0 && (c_den < 1 || c_num <= c_den || c_num > (1 << 20)))
        return fail(DSG_EINVAL, "the approximation ratio c = c_num / c_den must be > 1 (c_num <= 2^20)");
    const int tcap = T > 0 ? T : 1;
    const long long need = carve_par(n, nnz, tcap, nullptr, nullptr);
    if (workspace_bytes < need) return fail(DSG_EINVAL, "workspace too small (dsg_par_workspace_bytes)");
    DSG_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ParWs w;
    carve_par(n, nnz, tcap, static_cast<char*>(d_workspace), &w);
    hipStream_t s = ctx->stream;
    const int created_flags = 0;  // a cut of a valid graph is valid
    // one graph is bound at a time; it lives in this frame (no handle allocation)
    dsg_graph gb{};
    dsg_graph* g = nullptr;
    auto drop = [&]() {
        if (g) graph_fini(g);
        g = nullptr;
    };
    auto make = [&](int nn, long long mm, const int32_t* o, const int32_t* a) -> dsg_status {
        gb = dsg_graph();
        const dsg_status st = graph_init(&gb, ctx, nn, mm, o, a, w.gws, w.gws_bytes, tcap, created_flags, false);
        if (st == DSG_OK) g = &gb;
        return st;
    };
    auto bail = [&](dsg_status st) {
        drop();
        return st;
    };
    hipError_t e;
    int cur = 0, nc = 0, kmax = 0, level = 0, nrounds = 0;
    long long mc = 0;
    const int* cut_core = w.core;  // the core numbers (input ids) the cuts use
    dsg_par_apx apx{};
    dsg_status st;
    if (prune == 0) {
        // Coreness of the input graph (Coreness by buckets on the PEEL round loop),
        // then the ceil(k_max / 2)-core
        st = par_coreness(ctx, w, n, nnz, d_offsets, d_adj, tcap, flags, false, 0, 1, w.core, &gb, &g, &nrounds,
                          &kmax, nullptr);
        if (st != DSG_OK) return st;
        level = (kmax + 1) / 2;
        if ((e = dsg::launch_iota(w.iota, n, s)) != hipSuccess) return bail(hip_fail(e, "iota"));
        if ((st = par_cut(g, w, w.core, w.iota, level, cur, &nc, &mc)) != DSG_OK) return bail(st);
    } else {
        // the c-approximate decomposition (the round loop with eps = c - 1),
        // then the ceil(khat_max / 2c)-approximate core (Corollary apxkmax)
        st = par_coreness(ctx, w, n, nnz, d_offsets, d_adj, tcap, flags, false, c_num - c_den, c_den, w.apx, &gb,
                          &g, &nrounds, &apx.apx_kmax, nullptr);
        if (st != DSG_OK) return st;
        apx.apx_level = (int)(((long long)apx.apx_kmax * c_den + 2LL * c_num - 1) / (2LL * c_num));
        if ((e = dsg::launch_iota(w.iota, n, s)) != hipSuccess) return bail(hip_fail(e, "iota"));
        if ((st = par_cut(g, w, w.apx, w.iota, apx.apx_level, cur, &nc, &mc)) != DSG_OK) return bail(st);
        apx.apx_n = nc;
        apx.apx_nnz = mc;
        level = apx.apx_level;
        kmax = apx.apx_kmax;
        cut_core = w.apx;
        if (prune == 2) {
            // exact core numbers of the cut graph: at every level >= the
            // approximate one its cores are the input's
            drop();
            st = par_coreness(ctx, w, nc, mc, w.off[cur], w.adj[cur], tcap, created_flags, false, 0, 1, w.core1,
                              &gb, &g, &nrounds, &kmax, nullptr);
            if (st != DSG_OK) return st;
            if ((e = dsg::launch_scatter(w.core1, w.oldid[cur], nc, w.core, n, s)) != hipSuccess)
                return bail(hip_fail(e, "core numbers to input ids"));
            cut_core = w.core;
            // the exact max(L, ceil(k_max / 2))-core of the cut graph (it may
            // drop vertices even when the level stays: the approximate cut
            // keeps some vertices whose core number is below it)
            const int lv = (kmax + 1) / 2;
            if (lv > level) level = lv;
            int nn = 0;
            long long mm = 0;
            if ((st = par_cut(g, w, w.core, w.oldid[cur], level, 1 - cur, &nn, &mm)) != DSG_OK) return bail(st);
            cur = 1 - cur;
            nc = nn;
            mc = mm;
        }
    }
    if (((long long)T + 1) * (long long)g->d.max_deg >= (1LL << 31))
        return bail(fail(DSG_EOVERFLOW, "loads could exceed 31 bits: (T + 1) * max_degree >= 2^31"));
    drop();
    // S <- G: the first refined graph, loads zero
    if ((st = make(nc, mc, w.off[cur], w.adj[cur])) != DSG_OK) return st;
    long long be = mc / 2, bv = nc;
    int best_iter = 0, prunes = 0;
    if ((e = dsg::launch_vertex_mask(nc, w.oldid[cur], w.mask, n, s)) != hipSuccess) return bail(hip_fail(e, "mask"));
    for (int t = 1; t <= T; t++) {
        if ((st = dsg_run(g, 1, eps_num, eps_den, variant)) != DSG_OK) return bail(st);
        long long ie = 0, iv = 1;
        int ii = 0;
        const int slot = g->recorded - 1;
        DSG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        DSG_HIP(hipMemcpy(&ie, g->d.hist_e + slot, 8, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        DSG_HIP(hipMemcpy(&iv, g->d.hist_v + slot, 8, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        DSG_HIP(hipMemcpy(&ii, g->d.hist_i + slot, 4, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        if (h_iter_edges) h_iter_edges[t - 1] = ie;
        if (h_iter_verts) h_iter_verts[t - 1] = iv;
        if (h_iter_index) h_iter_index[t - 1] = ii;
        if (h_iter_n) h_iter_n[t - 1] = nc;
        if (h_iter_nnz) h_iter_nnz[t - 1] = mc / 2;
        if (h_iter_level) h_iter_level[t - 1] = level;
        // strict improvement by exact cross-multiplication (edges < 2^30, vertices < 2^26)
        if (ie * bv > be * iv) {
            be = ie;
            bv = iv;
            best_iter = t;
            if ((e = dsg::launch_suffix_mask(g->d, w.oldid[cur], ii, w.mask, n, s)) != hipSuccess)
                return bail(hip_fail(e, "mask"));
            const int lv = (int)((ie + iv - 1) / iv);  // ceil(rho(S))
            if (lv > level) {
                level = lv;
                prunes++;
                int nn = 0;
                long long mm = 0;
                if ((st = par_cut(g, w, cut_core, w.oldid[cur], level, 1 - cur, &nn, &mm)) != DSG_OK) return bail(st);
                const long long lb = g->load_bound;
                drop();
                cur = 1 - cur;
                nc = nn;
                mc = mm;
                if ((st = make(nc, mc, w.off[cur], w.adj[cur])) != DSG_OK) return st;
                // the surviving vertices keep their loads (graph creation zeroed them), and so does the bound
                // on them that sizes the SORT keys and the overflow guard
                DSG_HIP(hipMemcpyAsync(g->d.load, w.load, sizeof(int) * (size_t)nc, hipMemcpyDeviceToDevice, s),
                        "hipMemcpyAsync(loads)");
                g->load_bound = lb;
            }
        }
    }
    DSG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    result->best_edges = be;
    result->best_verts = bv;
    result->best_iter = best_iter;
    result->kmax = kmax;
    result->level = level;
    result->prunes = prunes;
    result->final_n = nc;
    result->final_nnz = mc;
    if (apx_out) *apx_out = apx;
    if (h_best_mask) DSG_HIP(hipMemcpy(h_best_mask, w.mask, (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy(mask)");
    if (h_core) DSG_HIP(hipMemcpy(h_core, cut_core, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy(core)");
    if (h_apx_core && prune != 0)
        DSG_HIP(hipMemcpy(h_apx_core, w.apx, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy(apx core)");
    drop();
    return DSG_OK;
}

}  // namespace

extern "C" {

dsg_status dsg_par_run(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                       void* d_workspace, int64_t workspace_bytes, int32_t T, int32_t eps_num, int32_t eps_den,
                       dsg_variant variant, int32_t flags, dsg_par_result* result, int64_t* h_iter_edges,
                       int64_t* h_iter_verts, int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz,
                       int32_t* h_iter_level, uint8_t* h_best_mask, int32_t* h_core) {
    return par_run_impl(ctx, n, nnz, d_offsets, d_adj, d_workspace, workspace_bytes, T, eps_num, eps_den, variant,
                        flags, 0, 1, 1, result, nullptr, h_iter_edges, h_iter_verts, h_iter_index, h_iter_n,
                        h_iter_nnz, h_iter_level, h_best_mask, h_core, nullptr);
}

dsg_status dsg_par_run_apx(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                           void* d_workspace, int64_t workspace_bytes, int32_t T, int32_t eps_num, int32_t eps_den,
                           dsg_variant variant, int32_t flags, int32_t then_exact, int32_t c_num, int32_t c_den,
                           dsg_par_result* result, dsg_par_apx* apx, int64_t* h_iter_edges, int64_t* h_iter_verts,
                           int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz, int32_t* h_iter_level,
                           uint8_t* h_best_mask, int32_t* h_core, int32_t* h_apx_core) {
    return par_run_impl(ctx, n, nnz, d_offsets, d_adj, d_workspace, workspace_bytes, T, eps_num, eps_den, variant,
                        flags, then_exact ? 2 : 1, c_num, c_den, result, apx, h_iter_edges, h_iter_verts,
                        h_iter_index, h_iter_n, h_iter_nnz, h_iter_level, h_best_mask, h_core, h_apx_core);
}

dsg_status dsg_par_run_noalloc(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                               int32_t T, int32_t eps_num, int32_t eps_den, dsg_variant variant, int32_t flags,
                               dsg_par_result* result, int64_t* h_iter_edges, int64_t* h_iter_verts,
                               int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz, int32_t* h_iter_level,
                               uint8_t* h_best_mask, int32_t* h_core) {
    if (!ctx) return fail(DSG_EINVAL, "NULL argument");
    if (n < 1 || n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "n must be in [1, 2^26)");
    if (nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "nnz must be in [0, 2^31 - 2^16]");
    if (T < 0) return fail(DSG_EINVAL, "T must be >= 0");
    const long long need = carve_par(n, nnz, T > 0 ? T : 1, nullptr, nullptr);
    if (need > DSG_NOALLOC_SCRATCH_BYTES) {
        char buf[192];
        snprintf(buf, sizeof buf, "graph needs %lld bytes of scratch; the static scratch holds %lld",
                 need, (long long)DSG_NOALLOC_SCRATCH_BYTES);
        return fail(DSG_ENOMEM, buf);
    }
    void* p = nullptr;
    hipError_t e = hipErrorInvalidDevice;
    if (ctx->device >= 0 && ctx->device < SCRATCH_MAX_DEVICES) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch_ptr[ctx->device];
        e = g_scratch_done[ctx->device] ? g_scratch_err[ctx->device] : hipErrorNotInitialized;
    }
    if (!p) return hip_fail(e, "static scratch address (hipGetSymbolAddress)");
    return par_run_impl(ctx, n, nnz, d_offsets, d_adj, p, DSG_NOALLOC_SCRATCH_BYTES, T, eps_num, eps_den, variant,
                        flags, 0, 1, 1, result, nullptr, h_iter_edges, h_iter_verts, h_iter_index, h_iter_n,
                        h_iter_nnz, h_iter_level, h_best_mask, h_core, nullptr);
}


}  // extern "C"

namespace {

long long al256(long long x) { return (x + 255) / 256 * 256; }

// Lays out the batch workspace: shared control data first, then each
// graph's arrays.  With base != nullptr the descriptors get real pointers.
long long carve_batch(const dsg_batch_graph* gr, int count, int t_cap, char* base, std::vector<dsg::BatchDesc>* out) {
    long long at = 0;
    const long long o_desc = at;
    at += al256(sizeof(dsg::BatchDesc) * (long long)count);
    const long long o_order = at;
    at += al256(4LL * count);
    const long long o_q = at;
    at += 256;
    const long long o_err = at;
    at += 256;
    const long long o_ctl = at;
    at += al256(sizeof(dsg::Ctl));
    if (out) out->resize(count);
    for (int g = 0; g < count; g++) {
        const long long n = gr[g].n, nch = gr[g].nnz / dsg::BATCH_MIN_CH + 2;
        dsg::BatchDesc d{};
        auto take = [&](long long bytes) {
            char* p = base ? base + at : nullptr;
            at += al256(bytes);
            return p;
        };
        d.load = (int*)take(4 * n);
        d.prio = (int*)take(4 * n);
        d.rnd = (int*)take(4 * n);
        d.inc = (int*)take(4 * n);
        d.pos = (int*)take(4 * n);
        d.L0 = (int*)take(4 * n);
        d.L1 = (int*)take(4 * n);
        d.iv = (int*)take(4 * n);
        d.ie = (int*)take(4 * n);
        d.ir = (int*)take(4 * n);
        d.A = (int*)take(4 * n);
        d.best_pos = (int*)take(4 * n);
        d.cfirst = (int*)take(4 * nch);
        d.clast = (int*)take(4 * nch);
        d.hist_e = (long long*)take(8LL * t_cap);
        d.hist_v = (long long*)take(8LL * t_cap);
        d.hist_i = (int*)take(4LL * t_cap);
        d.rounds = (int*)take(4LL * t_cap);
        d.digest = (unsigned long long*)take(8LL * t_cap);
        d.best = (long long*)take(32);
        d.state = (int*)take(32);
        d.n = gr[g].n;
        d.T = gr[g].T;
        d.eps_num = gr[g].eps_num;
        d.eps_den = gr[g].eps_den;
        d.nnz = gr[g].nnz;
        d.off = gr[g].d_offsets;
        d.adj = gr[g].d_adj;
        d.t_cap = t_cap;
        if (out) (*out)[g] = d;
    }
    (void)o_desc;
    (void)o_order;
    (void)o_q;
    (void)o_err;
    (void)o_ctl;
    return at;
}

dsg_status batch_index(dsg_batch* b, int i) {
    if (!b) return fail(DSG_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->count) return fail(DSG_EINVAL, "graph index out of range");
    return DSG_OK;
}

}  // namespace

extern "C" {

dsg_status dsg_batch_workspace_bytes(const dsg_batch_graph* graphs, int32_t count, int32_t t_cap, int64_t* bytes) {
    if (!graphs || !bytes || count < 1) return fail(DSG_EINVAL, "need graphs, count >= 1 and bytes");
    if (t_cap < 1) return fail(DSG_EINVAL, "t_cap must be >= 1");
    for (int g = 0; g < count; g++)
        if (graphs[g].n < 1 || graphs[g].nnz < 0 || graphs[g].nnz > dsg::MAX_NNZ)
            return fail(DSG_EINVAL, "graph " + std::to_string(g) + ": bad n or nnz");
    *bytes = carve_batch(graphs, count, t_cap, nullptr, nullptr);
    return DSG_OK;
}

dsg_status dsg_batch_create(dsg_ctx* ctx, const dsg_batch_graph* graphs, int32_t count, int32_t t_cap,
                            void* d_workspace, int64_t workspace_bytes, int32_t flags, dsg_batch** out) {
    if (!ctx || !graphs || !out || !d_workspace || count < 1) return fail(DSG_EINVAL, "NULL argument or count < 1");
    *out = nullptr;
    if (t_cap < 1) return fail(DSG_EINVAL, "t_cap must be >= 1");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(DSG_EINVAL, "workspace not 256-byte aligned");
    for (int g = 0; g < count; g++) {
        const dsg_batch_graph& x = graphs[g];
        if (x.n < 1 || x.nnz < 0 || x.nnz > dsg::MAX_NNZ || !x.d_offsets || (x.nnz > 0 && !x.d_adj))
            return fail(DSG_EINVAL, "graph " + std::to_string(g) + ": bad n, nnz or pointers");
        if (x.T < 0 || x.eps_num < 0 || x.eps_den < 1)
            return fail(DSG_EINVAL, "graph " + std::to_string(g) + ": bad T or eps");
        if (x.n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "graph " + std::to_string(g) + ": n too large");
    }
    const long long need = carve_batch(graphs, count, t_cap, nullptr, nullptr);
    if (workspace_bytes < need) return fail(DSG_ENOMEM, "workspace smaller than dsg_batch_workspace_bytes()");
    DSG_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    dsg_batch* b = new (std::nothrow) dsg_batch();
    if (!b) return fail(DSG_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    b->count = count;
    b->t_cap = t_cap;
    b->cfg = 0;
    b->blocks_per_cu = 4;
    char* base = static_cast<char*>(d_workspace);
    carve_batch(graphs, count, t_cap, base, &b->hdesc);
    b->ddesc = reinterpret_cast<dsg::BatchDesc*>(base);
    long long at = al256(sizeof(dsg::BatchDesc) * (long long)count);
    b->dorder = reinterpret_cast<int*>(base + at);
    at += al256(4LL * count);
    b->dqueue = reinterpret_cast<unsigned int*>(base + at);
    at += 256;
    b->derr = reinterpret_cast<int*>(base + at);
    at += 256;
    b->dctl = reinterpret_cast<dsg::Ctl*>(base + at);
    hipStream_t s = ctx->stream;
    auto bail = [&](dsg_status st) {
        delete b;
        return st;
    };
    // per-graph CSR checks, reusing the single-graph check kernels
    b->max_deg.assign(count, 0);
    b->iters.assign(count, 0);
    for (int g = 0; g < count; g++) {
        GraphDev gd{};
        gd.n = graphs[g].n;
        gd.nnz = graphs[g].nnz;
        gd.off = graphs[g].d_offsets;
        gd.adj = graphs[g].d_adj;
        gd.ctl = b->dctl;
        hipError_t e;
        if ((e = dsg::launch_zero_ctl(gd, s)) != hipSuccess) return bail(hip_fail(e, "zero ctl"));
        if ((e = dsg::launch_check_offsets(gd, s)) != hipSuccess) return bail(hip_fail(e, "check offsets"));
        dsg::Ctl c;
        if ((e = hipMemcpyAsync(&c, b->dctl, sizeof c, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return bail(hip_fail(e, "read checks"));
        if (c.err_count)
            return bail(fail(DSG_EINVAL, "graph " + std::to_string(g) + ": invalid CSR offsets"));
        if ((e = dsg::launch_check_range(gd, s)) != hipSuccess) return bail(hip_fail(e, "check range"));
        if ((flags & DSG_VALIDATE) && (e = dsg::launch_check_rows(gd, s)) != hipSuccess)
            return bail(hip_fail(e, "check rows"));
        if ((e = hipMemcpyAsync(&c, b->dctl, sizeof c, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return bail(hip_fail(e, "read checks"));
        if (c.err_count)
            return bail(fail(DSG_EINVAL, "graph " + std::to_string(g) + ": invalid CSR (" + err_name(c.err_code) + ")"));
        b->max_deg[g] = c.max_deg;
    }
    // largest first (longest-processing-time order), ties by index
    std::vector<int> order(count);
    for (int g = 0; g < count; g++) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return graphs[x].nnz > graphs[y].nnz; });
    hipError_t e;
    if ((e = hipMemcpyAsync(b->ddesc, b->hdesc.data(), sizeof(dsg::BatchDesc) * count, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(b->dorder, order.data(), 4LL * count, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(hip_fail(e, "upload descriptors"));
    if ((e = dsg::launch_batch_reset(b->ddesc, count, s)) != hipSuccess) return bail(hip_fail(e, "batch reset"));
    if ((e = dsg::launch_fill(b->derr, 0, 1, s)) != hipSuccess) return bail(hip_fail(e, "clear error flag"));
    if ((e = hipEventCreate(&b->ev0)) != hipSuccess) return bail(hip_fail(e, "hipEventCreate"));
    if ((e = hipEventCreate(&b->ev1)) != hipSuccess) {
        (void)hipEventDestroy(b->ev0);
        return bail(hip_fail(e, "hipEventCreate"));
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        (void)hipEventDestroy(b->ev0);
        (void)hipEventDestroy(b->ev1);
        return bail(hip_fail(e, "hipStreamSynchronize"));
    }
    *out = b;
    return DSG_OK;
}

dsg_status dsg_batch_set_config(dsg_batch* b, int32_t cfg, int32_t blocks_per_cu) {
    if (!b) return fail(DSG_EINVAL, "batch is NULL");
    if (cfg < 0 || cfg > 2 || blocks_per_cu < 1) return fail(DSG_EINVAL, "cfg must be 0..2 and blocks_per_cu >= 1");
    b->cfg = cfg;
    b->blocks_per_cu = blocks_per_cu;
    return DSG_OK;
}

dsg_status dsg_batch_run(dsg_batch* b) {
    if (!b) return fail(DSG_EINVAL, "batch is NULL");
    for (int g = 0; g < b->count; g++) {
        const dsg::BatchDesc& d = b->hdesc[g];
        if (b->iters[g] + d.T > b->t_cap)
            return fail(DSG_EINVAL, "graph " + std::to_string(g) + ": T exceeds the history capacity t_cap");
        if (((long long)b->iters[g] + d.T + 1) * (long long)b->max_deg[g] >= (1LL << 31))
            return fail(DSG_EOVERFLOW, "graph " + std::to_string(g) + ": loads could exceed 31 bits");
    }
    DSG_HIP(hipSetDevice(b->ctx->device), "hipSetDevice");
    hipStream_t s = b->ctx->stream;
    DSG_HIP(hipEventRecord(b->ev0, s), "hipEventRecord");
    hipError_t e = dsg::launch_batch(b->ddesc, b->dorder, b->count, b->dqueue, b->derr, b->cfg, b->blocks_per_cu,
                                     b->ctx->num_cu, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    DSG_HIP(hipEventRecord(b->ev1, s), "hipEventRecord");
    b->timed = true;
    for (int g = 0; g < b->count; g++) b->iters[g] += b->hdesc[g].T;
    return DSG_OK;
}

dsg_status dsg_batch_reset(dsg_batch* b) {
    if (!b) return fail(DSG_EINVAL, "batch is NULL");
    hipError_t e = dsg::launch_batch_reset(b->ddesc, b->count, b->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "batch reset");
    for (int g = 0; g < b->count; g++) b->iters[g] = 0;
    b->timed = false;
    return DSG_OK;
}

dsg_status dsg_batch_last_run_ms(dsg_batch* b, float* ms) {
    if (!b || !ms) return fail(DSG_EINVAL, "NULL argument");
    if (!b->timed) return fail(DSG_ESTATE, "no run recorded");
    DSG_HIP(hipEventSynchronize(b->ev1), "hipEventSynchronize");
    DSG_HIP(hipEventElapsedTime(ms, b->ev0, b->ev1), "hipEventElapsedTime");
    int err = 0;
    DSG_HIP(hipMemcpy(&err, b->derr, sizeof err, hipMemcpyDeviceToHost), "hipMemcpy(err)");
    if (err) return fail(DSG_EDEVICE, "a batch kernel consistency check failed");
    return DSG_OK;
}

dsg_status dsg_batch_get_best(dsg_batch* b, int32_t i, int64_t* edges, int64_t* verts, int32_t* iter, int32_t* index) {
    dsg_status st = batch_index(b, i);
    if (st != DSG_OK) return st;
    DSG_HIP(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    long long bs[4];
    DSG_HIP(hipMemcpy(bs, b->hdesc[i].best, sizeof bs, hipMemcpyDeviceToHost), "hipMemcpy(best)");
    if (edges) *edges = bs[0];
    if (verts) *verts = bs[1];
    if (iter) *iter = (int32_t)bs[2];
    if (index) *index = (int32_t)bs[3];
    return DSG_OK;
}

dsg_status dsg_batch_get_best_mask(dsg_batch* b, int32_t i, uint8_t* h_mask) {
    dsg_status st = batch_index(b, i);
    if (st != DSG_OK) return st;
    if (!h_mask) return fail(DSG_EINVAL, "mask is NULL");
    DSG_HIP(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    const dsg::BatchDesc& d = b->hdesc[i];
    long long bs[4];
    DSG_HIP(hipMemcpy(bs, d.best, sizeof bs, hipMemcpyDeviceToHost), "hipMemcpy(best)");
    if (bs[2] == 0) {
        memset(h_mask, 1, (size_t)d.n);
        return DSG_OK;
    }
    std::vector<int32_t> pos((size_t)d.n);
    DSG_HIP(hipMemcpy(pos.data(), d.best_pos, 4 * (size_t)d.n, hipMemcpyDeviceToHost), "hipMemcpy(best pos)");
    for (int v = 0; v < d.n; v++) h_mask[v] = pos[(size_t)v] >= bs[3] ? 1 : 0;
    return DSG_OK;
}

dsg_status dsg_batch_get_loads(dsg_batch* b, int32_t i, int64_t* h_loads) {
    dsg_status st = batch_index(b, i);
    if (st != DSG_OK) return st;
    if (!h_loads) return fail(DSG_EINVAL, "loads is NULL");
    DSG_HIP(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    const dsg::BatchDesc& d = b->hdesc[i];
    std::vector<int32_t> tmp((size_t)d.n);
    DSG_HIP(hipMemcpy(tmp.data(), d.load, 4 * (size_t)d.n, hipMemcpyDeviceToHost), "hipMemcpy(loads)");
    for (int v = 0; v < d.n; v++) h_loads[v] = tmp[(size_t)v];
    return DSG_OK;
}

dsg_status dsg_batch_get_iter_densities(dsg_batch* b, int32_t i, int64_t* h_edges, int64_t* h_verts, int32_t* h_index,
                                        int32_t cap, int32_t* count) {
    dsg_status st = batch_index(b, i);
    if (st != DSG_OK) return st;
    DSG_HIP(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    const dsg::BatchDesc& d = b->hdesc[i];
    const int rec = b->iters[i];
    const int k = cap < rec ? cap : rec;
    if (k > 0) {
        if (h_edges) DSG_HIP(hipMemcpy(h_edges, d.hist_e, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        if (h_verts) DSG_HIP(hipMemcpy(h_verts, d.hist_v, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
        if (h_index) DSG_HIP(hipMemcpy(h_index, d.hist_i, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(hist)");
    }
    if (count) *count = rec;
    return DSG_OK;
}

dsg_status dsg_batch_get_iter_digests(dsg_batch* b, int32_t i, uint64_t* h_digest, int32_t* h_rounds, int32_t cap,
                                      int32_t* count) {
    dsg_status st = batch_index(b, i);
    if (st != DSG_OK) return st;
    DSG_HIP(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    const dsg::BatchDesc& d = b->hdesc[i];
    const int rec = b->iters[i];
    const int k = cap < rec ? cap : rec;
    if (k > 0) {
        if (h_digest) DSG_HIP(hipMemcpy(h_digest, d.digest, 8 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(digest)");
        if (h_rounds) DSG_HIP(hipMemcpy(h_rounds, d.rounds, 4 * (size_t)k, hipMemcpyDeviceToHost), "hipMemcpy(rounds)");
    }
    if (count) *count = rec;
    return DSG_OK;
}

dsg_status dsg_batch_destroy(dsg_batch* b) {
    if (!b) return DSG_OK;
    (void)hipEventDestroy(b->ev0);
    (void)hipEventDestroy(b->ev1);
    delete b;
    return DSG_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- serving
namespace {

struct PoolAlloc {
    // first-fit free list over [0, size): offset -> length
    std::vector<std::pair<long long, long long>> free_list;
    void init(long long size) { free_list.assign(1, {0, size}); }
    long long alloc(long long bytes) {
        bytes = al256(bytes);
        for (size_t i = 0; i < free_list.size(); i++) {
            if (free_list[i].second >= bytes) {
                long long at = free_list[i].first;
                free_list[i].first += bytes;
                free_list[i].second -= bytes;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + (long)i);
                return at;
            }
        }
        return -1;
    }
    void release(long long at, long long bytes) {
        bytes = al256(bytes);
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(at, 0LL));
        it = free_list.insert(it, {at, bytes});
        // merge with neighbours
        size_t i = (size_t)(it - free_list.begin());
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + (long)i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + (long)i);
        }
    }
};

struct ServeReq {
    uint64_t ticket;
    long long at, bytes;  // the request's arrays in the pool
    dsg::BatchDesc d;
    bool reported;
    long long csr_at, csr_bytes;  // its CSR copy in the pool (0 bytes for a registered graph)
};

long long serve_footprint(int n, long long nnz, int T) {
    dsg_batch_graph g{};
    g.n = n;
    g.nnz = nnz;
    g.T = T;
    std::vector<dsg::BatchDesc> tmp;
    // the batch layout of one graph minus its shared header, plus the CSR
    const long long header = al256(sizeof(dsg::BatchDesc)) + 256 + 256 + 256 + al256(sizeof(dsg::Ctl));
    return carve_batch(&g, 1, T, nullptr, nullptr) - header + al256(4LL * (n + 1)) + al256(4LL * (nnz > 0 ? nnz : 1));
}

}  // namespace

struct dsg_server {
    dsg_ctx* ctx;
    char* pool;
    long long pool_bytes;
    int ring_size;
    dsg::ServeHostCtl* hctl;      // host view of the pinned control block
    dsg::ServeSlot* ring;         // host view of the pinned ring
    dsg::ServeHostCtl* hctl_dev;  // the same memory as the device addresses it
    dsg::ServeSlot* ring_dev;
    unsigned long long* dhead;
    int* derr;
    hipStream_t kstream, cstream;
    bool running;
    PoolAlloc alloc;
    uint64_t next_ticket;
    std::vector<ServeReq> reqs;  // in flight (admitted, not released)
    std::vector<char> slot_busy; // ring slot held by an unreleased request
    struct Reg {
        const int32_t* off;
        const int32_t* adj;
        int n;
        long long nnz;
        int max_deg;
    };
    std::vector<Reg> regs;       // resident graphs (caller-owned device CSR)
};

extern "C" {

dsg_status dsg_server_footprint(int32_t n, int64_t nnz, int32_t T, int64_t* bytes) {
    if (!bytes || n < 1 || nnz < 0 || nnz > dsg::MAX_NNZ || T < 1) return fail(DSG_EINVAL, "bad arguments");
    *bytes = serve_footprint(n, nnz, T);
    return DSG_OK;
}

dsg_status dsg_server_create(dsg_ctx* ctx, void* d_pool, int64_t pool_bytes, int32_t ring_size, dsg_server** out) {
    if (!ctx || !d_pool || !out || ring_size < 1 || pool_bytes < 4096) return fail(DSG_EINVAL, "bad arguments");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(d_pool) % 256 != 0) return fail(DSG_EINVAL, "pool not 256-byte aligned");
    DSG_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    dsg_server* s = new (std::nothrow) dsg_server();
    if (!s) return fail(DSG_ENOMEM, "host allocation failed");
    s->ctx = ctx;
    s->pool = static_cast<char*>(d_pool);
    s->pool_bytes = pool_bytes;
    s->ring_size = ring_size;
    // the first 512 bytes of the pool: claim counter and error flag
    s->dhead = reinterpret_cast<unsigned long long*>(s->pool);
    s->derr = reinterpret_cast<int*>(s->pool + 256);
    s->alloc.init(pool_bytes - 512);
    hipError_t e;
    void* hp = nullptr;
    if ((e = hipHostMalloc(&hp, sizeof(dsg::ServeHostCtl), hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess) {
        delete s;
        return hip_fail(e, "hipHostMalloc(ctl)");
    }
    s->hctl = static_cast<dsg::ServeHostCtl*>(hp);
    memset(s->hctl, 0, sizeof(dsg::ServeHostCtl));
    if ((e = hipHostMalloc(&hp, sizeof(dsg::ServeSlot) * (size_t)ring_size, hipHostMallocCoherent | hipHostMallocMapped)) !=
        hipSuccess) {
        (void)hipHostFree(s->hctl);
        delete s;
        return hip_fail(e, "hipHostMalloc(ring)");
    }
    s->ring = static_cast<dsg::ServeSlot*>(hp);
    memset(s->ring, 0, sizeof(dsg::ServeSlot) * (size_t)ring_size);
    s->slot_busy.assign((size_t)ring_size, 0);
    void* dp = nullptr;
    if ((e = hipHostGetDevicePointer(&dp, s->hctl, 0)) != hipSuccess) {
        (void)hipHostFree(s->ring);
        (void)hipHostFree(s->hctl);
        delete s;
        return hip_fail(e, "hipHostGetDevicePointer(ctl)");
    }
    s->hctl_dev = static_cast<dsg::ServeHostCtl*>(dp);
    if ((e = hipHostGetDevicePointer(&dp, s->ring, 0)) != hipSuccess) {
        (void)hipHostFree(s->ring);
        (void)hipHostFree(s->hctl);
        delete s;
        return hip_fail(e, "hipHostGetDevicePointer(ring)");
    }
    s->ring_dev = static_cast<dsg::ServeSlot*>(dp);
    if ((e = hipStreamCreateWithFlags(&s->kstream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking)) != hipSuccess) {
        (void)hipHostFree(s->ring);
        (void)hipHostFree(s->hctl);
        delete s;
        return hip_fail(e, "hipStreamCreate");
    }
    *out = s;
    return DSG_OK;
}

dsg_status dsg_server_start(dsg_server* s, int32_t cfg, int32_t blocks_per_cu, double idle_seconds, double max_seconds) {
    if (!s) return fail(DSG_EINVAL, "server is NULL");
    if (s->running) return fail(DSG_ESTATE, "already running");
    if (cfg < 0 || cfg > 1 || blocks_per_cu < 1 || !(idle_seconds > 0) || !(max_seconds > 0))
        return fail(DSG_EINVAL, "bad schedule or time limits");
    DSG_HIP(hipSetDevice(s->ctx->device), "hipSetDevice");
    __atomic_store_n(&s->hctl->shutdown, 0u, __ATOMIC_RELEASE);
    hipError_t e = dsg::launch_fill(s->derr, 0, 1, s->kstream);
    if (e != hipSuccess) return hip_fail(e, "clear error flag");
    const unsigned long long idle = (unsigned long long)(idle_seconds * 1e8);  // 100 MHz wall clock
    const unsigned long long maxt = (unsigned long long)(max_seconds * 1e8);
    // The claim counter restarts at the oldest published request that has
    // not finished.  A block always finishes the request it claimed before it
    // looks at the queue again, so once the previous kernel has exited every
    // claimed ticket is done and every unfinished one was never claimed: a
    // request published just as the last block left (after the submit's
    // running check) is run now instead of holding its ring slot and pool
    // regions for good.  Tickets are claimed in order, so the unfinished ones
    // are exactly [head0, tail).
    unsigned long long head0 = __atomic_load_n(&s->hctl->tail, __ATOMIC_ACQUIRE);
    for (const ServeReq& r : s->reqs) {
        const dsg::ServeSlot* sl = &s->ring[r.ticket % (uint64_t)s->ring_size];
        if (__atomic_load_n(&sl->done, __ATOMIC_ACQUIRE) != r.ticket + 1 && r.ticket < head0) head0 = r.ticket;
    }
    e = dsg::launch_serve(s->hctl_dev, s->ring_dev, s->ring_size, s->dhead, head0, s->derr, cfg, blocks_per_cu,
                          s->ctx->num_cu, idle, maxt, s->kstream);
    if (e != hipSuccess) return hip_fail(e, "serve launch");
    s->running = true;
    return DSG_OK;
}

}  // extern "C"

namespace {

// Admit one request whose CSR is at d_off/d_adj on the device (copied by the
// caller of this function if it came from the host): reserve its arrays in
// the pool, fill its ring slot and publish it.  extra_bytes/extra_at: a
// pool region already reserved for the CSR copy (freed with the request).
dsg_status serve_publish(dsg_server* s, const int32_t* d_off, const int32_t* d_adj, int n, long long nnz, int T,
                         int eps_num, int eps_den, long long extra_at, long long extra_bytes, uint64_t* ticket) {
    const long long header = al256(sizeof(dsg::BatchDesc)) + 256 + 256 + 256 + al256(sizeof(dsg::Ctl));
    dsg_batch_graph g{};
    g.d_offsets = d_off;
    g.d_adj = d_adj;
    g.n = n;
    g.nnz = nnz;
    g.T = T;
    g.eps_num = eps_num;
    g.eps_den = eps_den;
    const long long bytes = carve_batch(&g, 1, T, nullptr, nullptr) - header;
    const long long at = s->alloc.alloc(bytes);
    if (at < 0) {
        if (extra_bytes) s->alloc.release(extra_at, extra_bytes);
        return fail(DSG_EBUSY, "HBM pool full");
    }
    std::vector<dsg::BatchDesc> desc;
    carve_batch(&g, 1, T, s->pool + 512 + at - header, &desc);
    const uint64_t t = s->next_ticket++;
    dsg::ServeSlot* sl = &s->ring[t % (uint64_t)s->ring_size];
    sl->d = desc[0];
    __atomic_store_n(&sl->done, 0ull, __ATOMIC_RELAXED);
    __atomic_store_n(&s->hctl->tail, (unsigned long long)(t + 1), __ATOMIC_RELEASE);
    s->reqs.push_back(ServeReq{t, at, bytes, desc[0], false, extra_at, extra_bytes});
    s->slot_busy[(size_t)(t % (uint64_t)s->ring_size)] = 1;
    *ticket = t;
    return DSG_OK;
}

dsg_status serve_precheck(dsg_server* s, int T, int eps_num, int eps_den, int maxdeg) {
    if (T < 1 || eps_num < 0 || eps_den < 1) return fail(DSG_EINVAL, "bad T or eps");
    if (!s->running || hipStreamQuery(s->kstream) == hipSuccess) {
        s->running = false;
        return fail(DSG_ESTATE, "server kernel is not running");
    }
    if (((long long)T + 1) * (long long)maxdeg >= (1LL << 31)) return fail(DSG_EOVERFLOW, "loads could exceed 31 bits");
    // ticket t lives in ring slot t % ring_size: that slot must be free
    if (s->slot_busy[(size_t)(s->next_ticket % (uint64_t)s->ring_size)])
        return fail(DSG_EBUSY, "the next ring slot is still held by an unreleased request");
    return DSG_OK;
}

}  // namespace

extern "C" {

dsg_status dsg_server_submit(dsg_server* s, const int32_t* h_off, const int32_t* h_adj, int32_t n, int64_t nnz,
                             int32_t T, int32_t eps_num, int32_t eps_den, uint64_t* ticket) {
    if (!s || !h_off || !ticket || (nnz > 0 && !h_adj)) return fail(DSG_EINVAL, "NULL argument");
    if (n < 1 || nnz < 0 || nnz > dsg::MAX_NNZ) return fail(DSG_EINVAL, "bad n or nnz");
    if (n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "n too large");
    // memory-safety checks of the CSR on the host: offsets and entry range
    if (h_off[0] != 0 || (long long)h_off[n] != nnz) return fail(DSG_EINVAL, "offsets[0] != 0 or offsets[n] != nnz");
    int maxdeg = 0;
    for (int v = 0; v < n; v++) {
        const int d = h_off[v + 1] - h_off[v];
        if (d < 0) return fail(DSG_EINVAL, "offsets decrease");
        if (d > maxdeg) maxdeg = d;
    }
    for (long long e = 0; e < nnz; e++)
        if (h_adj[e] < 0 || h_adj[e] >= n) return fail(DSG_EINVAL, "adjacency entry outside [0, n)");
    dsg_status st = serve_precheck(s, T, eps_num, eps_den, maxdeg);
    if (st != DSG_OK) return st;
    const long long csr_bytes = al256(4LL * (n + 1)) + al256(4LL * (nnz > 0 ? nnz : 1));
    const long long cat = s->alloc.alloc(csr_bytes);
    if (cat < 0) return fail(DSG_EBUSY, "HBM pool full");
    int32_t* d_off = reinterpret_cast<int32_t*>(s->pool + 512 + cat);
    int32_t* d_adj = reinterpret_cast<int32_t*>(s->pool + 512 + cat + al256(4LL * (n + 1)));
    hipError_t e = hipMemcpyAsync(d_off, h_off, 4LL * (n + 1), hipMemcpyHostToDevice, s->cstream);
    if (e == hipSuccess && nnz > 0) e = hipMemcpyAsync(d_adj, h_adj, 4LL * nnz, hipMemcpyHostToDevice, s->cstream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->cstream);
    if (e != hipSuccess) {
        s->alloc.release(cat, csr_bytes);
        return hip_fail(e, "copy request CSR");
    }
    return serve_publish(s, d_off, d_adj, n, nnz, T, eps_num, eps_den, cat, csr_bytes, ticket);
}

dsg_status dsg_server_register(dsg_server* s, const int32_t* d_offsets, const int32_t* d_adj, int32_t n, int64_t nnz,
                               int32_t flags, int32_t* graph_id) {
    if (!s || !d_offsets || !graph_id || (nnz > 0 && !d_adj)) return fail(DSG_EINVAL, "NULL argument");
    if (n < 1 || nnz < 0 || nnz > dsg::MAX_NNZ || n >= dsg::PEEL_MAX_N) return fail(DSG_EINVAL, "bad n or nnz");
    if (s->running) return fail(DSG_ESTATE, "register graphs before dsg_server_start");
    // device checks with the single-graph check kernels, on the copy stream;
    // the control block sits in the pool's reserved header
    GraphDev gd{};
    gd.n = n;
    gd.nnz = nnz;
    gd.off = d_offsets;
    gd.adj = d_adj;
    // borrow a pool region for a control block
    const long long cat = s->alloc.alloc(sizeof(dsg::Ctl));
    if (cat < 0) return fail(DSG_EBUSY, "HBM pool full");
    gd.ctl = reinterpret_cast<dsg::Ctl*>(s->pool + 512 + cat);
    hipStream_t c = s->cstream;
    dsg::Ctl ctl;
    hipError_t e = dsg::launch_zero_ctl(gd, c);
    if (e == hipSuccess) e = dsg::launch_check_offsets(gd, c);
    if (e == hipSuccess) e = hipMemcpyAsync(&ctl, gd.ctl, sizeof ctl, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess) e = hipStreamSynchronize(c);
    if (e == hipSuccess && ctl.err_count == 0) {
        e = dsg::launch_check_range(gd, c);
        if (e == hipSuccess && (flags & DSG_VALIDATE)) e = dsg::launch_check_rows(gd, c);
        if (e == hipSuccess) e = hipMemcpyAsync(&ctl, gd.ctl, sizeof ctl, hipMemcpyDeviceToHost, c);
        if (e == hipSuccess) e = hipStreamSynchronize(c);
    }
    s->alloc.release(cat, sizeof(dsg::Ctl));
    if (e != hipSuccess) return hip_fail(e, "check registered graph");
    if (ctl.err_count) return fail(DSG_EINVAL, std::string("invalid CSR (") + err_name(ctl.err_code) + ")");
    s->regs.push_back(dsg_server::Reg{d_offsets, d_adj, n, nnz, ctl.max_deg});
    *graph_id = (int32_t)s->regs.size() - 1;
    return DSG_OK;
}

dsg_status dsg_server_submit_registered(dsg_server* s, int32_t graph_id, int32_t T, int32_t eps_num, int32_t eps_den,
                                        uint64_t* ticket) {
    if (!s || !ticket) return fail(DSG_EINVAL, "NULL argument");
    if (graph_id < 0 || graph_id >= (int)s->regs.size()) return fail(DSG_EINVAL, "unknown graph id");
    const dsg_server::Reg& r = s->regs[(size_t)graph_id];
    dsg_status st = serve_precheck(s, T, eps_num, eps_den, r.max_deg);
    if (st != DSG_OK) return st;
    return serve_publish(s, r.off, r.adj, r.n, r.nnz, T, eps_num, eps_den, 0, 0, ticket);
}

dsg_status dsg_server_poll(dsg_server* s, uint64_t* h_tickets, int32_t cap, int32_t* count) {
    if (!s || !count) return fail(DSG_EINVAL, "NULL argument");
    int k = 0;
    for (ServeReq& r : s->reqs) {
        if (k >= cap) break;
        if (r.reported) continue;
        const dsg::ServeSlot* sl = &s->ring[r.ticket % (uint64_t)s->ring_size];
        if (__atomic_load_n(&sl->done, __ATOMIC_ACQUIRE) == r.ticket + 1) {
            r.reported = true;
            if (h_tickets) h_tickets[k] = r.ticket;
            k++;
        }
    }
    *count = k;
    return DSG_OK;
}

dsg_status dsg_server_fetch(dsg_server* s, uint64_t ticket, int64_t* best, int64_t* h_edges, int64_t* h_verts,
                            int32_t* h_index, uint64_t* h_digest, int32_t* h_rounds, int64_t* h_loads) {
    if (!s) return fail(DSG_EINVAL, "server is NULL");
    ServeReq* r = nullptr;
    for (ServeReq& x : s->reqs)
        if (x.ticket == ticket) r = &x;
    if (!r) return fail(DSG_EINVAL, "unknown ticket");
    const dsg::ServeSlot* sl = &s->ring[ticket % (uint64_t)s->ring_size];
    if (__atomic_load_n(&sl->done, __ATOMIC_ACQUIRE) != ticket + 1) return fail(DSG_ESTATE, "request not finished");
    const dsg::BatchDesc& d = r->d;
    const int T = d.T;
    hipStream_t c = s->cstream;
    long long bs[4];
    std::vector<int32_t> loads32;
    hipError_t e = hipMemcpyAsync(bs, d.best, sizeof bs, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_edges) e = hipMemcpyAsync(h_edges, d.hist_e, 8LL * T, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_verts) e = hipMemcpyAsync(h_verts, d.hist_v, 8LL * T, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_index) e = hipMemcpyAsync(h_index, d.hist_i, 4LL * T, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_digest) e = hipMemcpyAsync(h_digest, d.digest, 8LL * T, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_rounds) e = hipMemcpyAsync(h_rounds, d.rounds, 4LL * T, hipMemcpyDeviceToHost, c);
    if (e == hipSuccess && h_loads) {
        loads32.resize((size_t)d.n);
        e = hipMemcpyAsync(loads32.data(), d.load, 4LL * d.n, hipMemcpyDeviceToHost, c);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c);
    if (e != hipSuccess) return hip_fail(e, "fetch results");
    if (best)
        for (int i = 0; i < 4; i++) best[i] = bs[i];
    if (h_loads)
        for (int v = 0; v < d.n; v++) h_loads[v] = loads32[(size_t)v];
    return DSG_OK;
}

dsg_status dsg_server_release(dsg_server* s, uint64_t ticket) {
    if (!s) return fail(DSG_EINVAL, "server is NULL");
    for (size_t i = 0; i < s->reqs.size(); i++) {
        if (s->reqs[i].ticket != ticket) continue;
        const dsg::ServeSlot* sl = &s->ring[ticket % (uint64_t)s->ring_size];
        if (__atomic_load_n(&sl->done, __ATOMIC_ACQUIRE) != ticket + 1)
            return fail(DSG_ESTATE, "request not finished");
        s->alloc.release(s->reqs[i].at, s->reqs[i].bytes);
        if (s->reqs[i].csr_bytes) s->alloc.release(s->reqs[i].csr_at, s->reqs[i].csr_bytes);
        s->slot_busy[(size_t)(ticket % (uint64_t)s->ring_size)] = 0;
        s->reqs.erase(s->reqs.begin() + (long)i);
        return DSG_OK;
    }
    return fail(DSG_EINVAL, "unknown ticket");
}

dsg_status dsg_server_stop(dsg_server* s) {
    if (!s) return fail(DSG_EINVAL, "server is NULL");
    __atomic_store_n(&s->hctl->shutdown, 1u, __ATOMIC_RELEASE);
    DSG_HIP(hipStreamSynchronize(s->kstream), "hipStreamSynchronize(server)");
    s->running = false;
    int err = 0;
    DSG_HIP(hipMemcpy(&err, s->derr, sizeof err, hipMemcpyDeviceToHost), "hipMemcpy(err)");
    if (err) return fail(DSG_EDEVICE, "a serving kernel consistency check failed");
    return DSG_OK;
}

dsg_status dsg_server_destroy(dsg_server* s) {
    if (!s) return DSG_OK;
    if (s->running) {
        __atomic_store_n(&s->hctl->shutdown, 1u, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(s->kstream);
    }
    (void)hipStreamDestroy(s->kstream);
    (void)hipStreamDestroy(s->cstream);
    (void)hipHostFree(s->ring);
    (void)hipHostFree(s->hctl);
    delete s;
    return DSG_OK;
}

}  // extern "C"
