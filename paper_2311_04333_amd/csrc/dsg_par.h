// dsg_par.h -- kernels of the Pruning-and-Refining framework (Algorithm 1,
// Section 3): core numbers and core-subgraph extraction.  Internal.
#pragma once

#include "dsg_internal.h"

namespace dsg {

// Exclusive-scan scratch: one int64 per 4096-element tile.
long long par_scan_tiles(long long count);

// Core numbers from a finished PEEL iteration run with zero loads and
// monotone thresholds on graph `g`: round r peels every alive vertex whose
// degree is at most D_r = max(D_{r-1}, floor((1 + eps) * round minimum)),
// and core(v) = D at v's round.  With eps = 0 these are the exact core
// numbers (Coreness, Section 2, by buckets); with eps > 0 they are a
// (1 + eps)-approximate decomposition with core <= khat <= (1 + eps) core.
// `rv` holds the round bounds, written by the round loop (GraphDev::rmin);
// their running maximum is taken in place (they are already monotone).
// Writes core[0..n) and *kmax_dev (one int).
hipError_t launch_core_numbers(const GraphDev& g, int nrounds, int* rv, int* core, int* kmax_dev, hipStream_t s);

// Subgraph of the current graph `g` induced by {x : core[oldid[x]] >= level}
// (getCore, Algorithm 1), ids renumbered in order.  Device outputs:
// new_off[0..n_new], new_adj, new_oldid[n_new] (input-graph ids) and
// new_load[n_new] (the current loads carried over), plus *counts_dev =
// {n_new, nnz_new} (two int64).  Scratch: keep/newid (n + 1 ints each),
// f/fs (nnz + 1 ints each), tiles (par_scan_tiles(max(n, nnz) + 1)
// int64).  The static item list of `g` must be built (graph creation does).
struct CoreCut {
    const int* oldid;
    const int* core;
    int level;
    int* keep;
    int* newid;
    int* f;
    int* fs;
    long long* tiles;
    int* new_off;
    int* new_adj;
    int* new_oldid;
    int* new_load;
    long long* counts_dev;
};
hipError_t launch_get_core(const GraphDev& g, const CoreCut& c, hipStream_t s);

// mask[oldid[order[i]]] = 1 for i >= idx (the iteration's densest suffix, in
// input ids); mask is zeroed first (n_input bytes).
hipError_t launch_suffix_mask(const GraphDev& g, const int* oldid, int idx, unsigned char* mask, long long n_input,
                              hipStream_t s);

// mask[oldid[x]] = 1 for every vertex x of a graph with n vertices.
hipError_t launch_vertex_mask(int n, const int* oldid, unsigned char* mask, long long n_input, hipStream_t s);

// out[i] = i for i < n.
hipError_t launch_iota(int* out, int n, hipStream_t s);

// dst[0..n_dst) = 0, then dst[idx[x]] = src[x] for x < n_src (core numbers of
// a cut graph, moved to input ids).
hipError_t launch_scatter(const int* src, const int* idx, int n_src, int* dst, long long n_dst, hipStream_t s);

}  // namespace dsg
