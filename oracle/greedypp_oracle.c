/*
 * greedypp_oracle.c -- plain CPU oracle for the Greedy++ peeling hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * Written from Sukprasert, Liu, Dhulipala, Shun, "Practical Parallel
 * Algorithms for Near-Optimal Densest Subgraphs on Massive Graphs"
 * (arXiv 2311.04333).  Everything is exact integer arithmetic; products that
 * compare rationals use 128-bit integers so that no overflow is possible.
 *
 * What one iteration computes (all variants), given loads l(v) fixed for the
 * iteration:
 *   1. an ordering v_1..v_n of the vertices (the variant decides it);
 *   2. Algorithm 3 (Section 3.3): every edge (v_j, v_k) adds one to
 *      A[min(j,k)]; B = SuffixSum(A); the prefix-removed subgraph
 *      S_i = {v_i..v_n} has |E(S_i)| = B[i] and |S_i| = n-i+1 vertices; the
 *      iteration's best density is max_i B[i]/(n-i+1); loads grow by
 *      l(v_i) += A[i].
 *   3. the running best subgraph S is replaced only on a strictly larger
 *      density (Algorithm 2 compares rho(H) > rho(S), starting from S = G).
 * Indices below are 0-based: candidate i is S_i = {v : pos[v] >= i}, of size
 * n-i; ties between candidates go to the smallest i (the first one Algorithm 2
 * would meet while peeling).
 *
 * Orderings:
 *   SEQ  -- the load ordering of Section 2: repeatedly peel the alive vertex
 *           minimising l(v) + deg(v) (current induced degree); ties -> lower id.
 *           With l = 0 this is the degeneracy ordering (Coreness).
 *   PEEL -- round-synchronous peeling (the parallel ordering of Section 3.3,
 *           "ParallelGreedy++", with the round rule parameterised by eps):
 *           each round takes mn = min over alive of l(v)+deg(v) and peels every
 *           alive v with l(v)+deg(v) <= (1+eps) mn, eps = eps_num/eps_den.  All
 *           vertices of a round see the degrees of the round's start (their
 *           mutual effects are delayed to the end of the step).  Within a round
 *           positions follow ascending vertex id, so a same-round edge is
 *           charged to its lower-id endpoint.
 *   SORT -- GreedySorting++ (Section 3.2): sort by the load at the start of the
 *           iteration, ascending, ties -> lower id.
 *   PEEL_MONO -- PEEL with the bucketing of the exact k-core algorithm the
 *           paper uses (Section 3.1, Julienne): a bucket bound d only grows.
 *           Round r peels every alive v with l(v)+deg(v) <= d_r, where
 *           d_r = max(d_{r-1}, (1+eps) mn_r) and d_{-1} = -infinity; with
 *           eps = 0 and zero loads this is "peel everything of degree at
 *           most d, raise d when nothing is left at or below it".  d starts
 *           afresh in every iteration.
 *
 * The fused form (orc_run_fused) is Algorithm 2 as printed: it keeps |E(H)|
 * and |V(H)| while peeling one vertex at a time and charges each vertex its
 * degree at the moment it is peeled.  It shares no bookkeeping with the
 * decoupled form (ordering, then Algorithm 3), and tests require the two to
 * agree exactly.
 *
 * Digest of an ordering: sum over v of mix64((v << 32) | (uint32)round[v])
 * mod 2^64, where mix64 is the SplitMix64 output function (Steele, Lea,
 * Flood 2014) and round[v] is the peeling round (PEEL) or the position
 * (SEQ, SORT).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;
typedef uint64_t u64;
typedef __int128 i128;

enum { ORC_SEQ = 0, ORC_PEEL = 1, ORC_SORT = 2, ORC_PEEL_MONO = 3 };

static u64 orc_mix64(u64 z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

u64 orc_digest(int32_t n, const int32_t* round) {
    u64 s = 0;
    for (int32_t v = 0; v < n; v++) s += orc_mix64(((u64)(uint32_t)v << 32) | (u64)(uint32_t)round[v]);
    return s;
}

/* ------------------------------------------------------------ orderings */

/* SEQ: n single-vertex steps, each an O(n) scan for the minimum of
 * (l(v) + deg(v), v) over alive vertices.  Returns the number of steps (n). */
int32_t orc_order_seq(int32_t n, const int32_t* off, const int32_t* adj, const i64* load, int32_t* pos,
                      int32_t* round) {
    i64* deg = (i64*)malloc(sizeof(i64) * (size_t)n);
    char* alive = (char*)malloc((size_t)n);
    if (!deg || !alive) {
        free(deg);
        free(alive);
        return -1;
    }
    for (int32_t v = 0; v < n; v++) {
        deg[v] = off[v + 1] - off[v];
        alive[v] = 1;
    }
    for (int32_t j = 0; j < n; j++) {
        int32_t best = -1;
        for (int32_t v = 0; v < n; v++) {
            if (!alive[v]) continue;
            if (best < 0 || load[v] + deg[v] < load[best] + deg[best]) best = v;
        }
        pos[best] = j;
        round[best] = j;
        alive[best] = 0;
        for (int32_t k = off[best]; k < off[best + 1]; k++)
            if (alive[adj[k]]) deg[adj[k]]--;
    }
    free(deg);
    free(alive);
    return n;
}

/* PEEL: round-synchronous (1+eps)-of-minimum peeling.  The alive list is kept
 * in ascending id order, so each round's frontier comes out in ascending id.
 * With `mono`, the bound of a round is the largest bound of the iteration so
 * far (PEEL_MONO).  Returns the number of rounds. */
int32_t orc_order_peel_rule(int32_t n, const int32_t* off, const int32_t* adj, const i64* load, i64 eps_num,
                            i64 eps_den, int32_t mono, int32_t* pos, int32_t* round) {
    i64* deg = (i64*)malloc(sizeof(i64) * (size_t)n);
    int32_t* alive = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !alive) {
        free(deg);
        free(alive);
        return -1;
    }
    for (int32_t v = 0; v < n; v++) {
        deg[v] = off[v + 1] - off[v];
        round[v] = -1;
        alive[v] = v;
    }
    int32_t nalive = n, r = 0, next = 0;
    i128 dmax = -1; /* largest bound so far, scaled by eps_den (PEEL_MONO) */
    while (nalive > 0) {
        /* minimum priority over the alive vertices */
        i64 mn = load[alive[0]] + deg[alive[0]];
        for (int32_t k = 1; k < nalive; k++) {
            i64 p = load[alive[k]] + deg[alive[k]];
            if (p < mn) mn = p;
        }
        /* frontier: every alive v with eps_den * p(v) <= (eps_den + eps_num) * mn
         * (or the larger earlier bound, PEEL_MONO), selected with the degrees
         * of the round's start, in ascending id */
        i128 lim = (i128)(eps_den + eps_num) * (i128)mn;
        if (mono) {
            if (dmax > lim) lim = dmax;
            dmax = lim;
        }
        for (int32_t k = 0; k < nalive; k++) {
            int32_t v = alive[k];
            if ((i128)eps_den * (i128)(load[v] + deg[v]) <= lim) {
                round[v] = r;
                pos[v] = next++;
            }
        }
        /* delayed effects: each peeled vertex removes one from every neighbour
         * that survives the round */
        for (int32_t k = 0; k < nalive; k++) {
            int32_t v = alive[k];
            if (round[v] != r) continue;
            for (int32_t e = off[v]; e < off[v + 1]; e++)
                if (round[adj[e]] == -1) deg[adj[e]]--;
        }
        int32_t keep = 0;
        for (int32_t k = 0; k < nalive; k++)
            if (round[alive[k]] == -1) alive[keep++] = alive[k];
        nalive = keep;
        r++;
    }
    free(deg);
    free(alive);
    return r;
}

int32_t orc_order_peel(int32_t n, const int32_t* off, const int32_t* adj, const i64* load, i64 eps_num, i64 eps_den,
                       int32_t* pos, int32_t* round) {
    return orc_order_peel_rule(n, off, adj, load, eps_num, eps_den, 0, pos, round);
}

/* SORT: ids ordered by (load, id) ascending.  qsort on packed pairs. */
typedef struct {
    i64 key;
    int32_t id;
} kv;

static int kv_cmp(const void* a, const void* b) {
    const kv* x = (const kv*)a;
    const kv* y = (const kv*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

int32_t orc_order_sort(int32_t n, const i64* load, int32_t* pos, int32_t* round) {
    kv* a = (kv*)malloc(sizeof(kv) * (size_t)n);
    if (!a) return -1;
    for (int32_t v = 0; v < n; v++) {
        a[v].key = load[v];
        a[v].id = v;
    }
    qsort(a, (size_t)n, sizeof(kv), kv_cmp);
    for (int32_t i = 0; i < n; i++) {
        pos[a[i].id] = i;
        round[a[i].id] = i;
    }
    free(a);
    return n;
}

/* --------------------------------------------------------- Algorithm 3 */

/* Charges A[min(pos u, pos v)] += 1 for every undirected edge, forms the suffix
 * sums B, and returns the iteration's best candidate (edges, vertices, index)
 * with ties to the smallest index.  A and B are caller arrays of length n. */
void orc_alg3(int32_t n, const int32_t* off, const int32_t* adj, const int32_t* pos, i64* A, i64* B, i64* it_e,
              i64* it_v, i64* it_i) {
    memset(A, 0, sizeof(i64) * (size_t)n);
    for (int32_t u = 0; u < n; u++)
        for (int32_t e = off[u]; e < off[u + 1]; e++) {
            int32_t v = adj[e];
            if (u < v) A[pos[u] < pos[v] ? pos[u] : pos[v]] += 1; /* each edge once */
        }
    i64 run = 0;
    for (int32_t i = n - 1; i >= 0; i--) {
        run += A[i];
        B[i] = run;
    }
    i64 be = B[0], bv = n, bi = 0;
    for (int32_t i = 1; i < n; i++) {
        i64 e = B[i], v = n - i;
        if ((i128)e * bv > (i128)be * v) {
            be = e;
            bv = v;
            bi = i;
        }
    }
    *it_e = be;
    *it_v = bv;
    *it_i = bi;
}

/* ------------------------------------------------------------- full runs */

/* State carried between calls (so that run(a) then run(b) equals run(a+b)):
 *   load[n]        int64 loads
 *   best[4]        (edges, vertices, iteration, index) of the best subgraph;
 *                  initialise to (m, n, 0, 0): S = G
 *   best_pos[n]    positions of the iteration that produced best (its vertex
 *                  set is {v : best_pos[v] >= best index}); untouched while
 *                  best iteration is 0
 *   iter_done      iterations already performed (numbering continues)
 * Per-iteration outputs for t = 0..T-1 of this call:
 *   hist[2t], hist[2t+1]  the iteration's best (edges, vertices)
 *   hist_idx[t]           its index
 *   digest[t]             ordering digest
 *   nrounds[t]            rounds (PEEL) or n
 *   width[t]              max over v of the load increase (empirical width)
 * Last iteration: last_pos[n], last_round[n].
 * Returns 0, or -1 on allocation failure / bad arguments. */
int orc_run(int32_t n, const int32_t* off, const int32_t* adj, int32_t T, int32_t variant, i64 eps_num, i64 eps_den,
            i64* load, i64* best, int32_t* best_pos, int32_t iter_done, i64* hist, i64* hist_idx, u64* digest,
            int32_t* nrounds, i64* width, int32_t* last_pos, int32_t* last_round) {
    if (n < 1 || T < 0 || eps_num < 0 || eps_den < 1) return -1;
    i64* A = (i64*)malloc(sizeof(i64) * (size_t)n);
    i64* B = (i64*)malloc(sizeof(i64) * (size_t)n);
    if (!A || !B) {
        free(A);
        free(B);
        return -1;
    }
    for (int32_t t = 0; t < T; t++) {
        int32_t rounds;
        if (variant == ORC_SEQ)
            rounds = orc_order_seq(n, off, adj, load, last_pos, last_round);
        else if (variant == ORC_PEEL || variant == ORC_PEEL_MONO)
            rounds = orc_order_peel_rule(n, off, adj, load, eps_num, eps_den, variant == ORC_PEEL_MONO, last_pos,
                                         last_round);
        else
            rounds = orc_order_sort(n, load, last_pos, last_round);
        if (rounds < 0) {
            free(A);
            free(B);
            return -1;
        }
        i64 e, v, i;
        orc_alg3(n, off, adj, last_pos, A, B, &e, &v, &i);
        i64 w = 0;
        for (int32_t u = 0; u < n; u++) {
            i64 inc = A[last_pos[u]];
            load[u] += inc;
            if (inc > w) w = inc;
        }
        hist[2 * t] = e;
        hist[2 * t + 1] = v;
        hist_idx[t] = i;
        digest[t] = orc_digest(n, last_round);
        nrounds[t] = rounds;
        width[t] = w;
        if ((i128)e * best[1] > (i128)best[0] * v) {
            best[0] = e;
            best[1] = v;
            best[2] = iter_done + t + 1;
            best[3] = i;
            memcpy(best_pos, last_pos, sizeof(int32_t) * (size_t)n);
        }
    }
    free(A);
    free(B);
    return 0;
}

/* Algorithm 2 in its fused form.  The peel sequence is generated on the fly:
 *   SEQ  -- argmin of (l(v) + deg_H(v), v) among vertices still in H;
 *   PEEL -- rounds as in orc_order_peel, but each frontier vertex is removed
 *           from H one at a time (ascending id), so it is charged its degree
 *           in H at that moment;
 *   SORT -- the (load, id) order fixed at the iteration's start.
 * Before each single peel the density of H is compared with the best so far
 * (strict), and the iteration's own maximum is tracked with the same rule.
 * Outputs as for orc_run (no digest/rounds/width); last_pos gets positions. */
int orc_run_fused(int32_t n, const int32_t* off, const int32_t* adj, int32_t T, int32_t variant, i64 eps_num,
                  i64 eps_den, i64* load, i64* best, int32_t* best_pos, int32_t iter_done, i64* hist, i64* hist_idx,
                  int32_t* last_pos) {
    if (n < 1 || T < 0 || eps_num < 0 || eps_den < 1) return -1;
    i64* degH = (i64*)malloc(sizeof(i64) * (size_t)n);
    i64* start = (i64*)malloc(sizeof(i64) * (size_t)n); /* loads at iteration start */
    char* inH = (char*)malloc((size_t)n);
    int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    char* inF = (char*)malloc((size_t)n);
    if (!degH || !start || !inH || !seq || !inF) {
        free(degH); free(start); free(inH); free(seq); free(inF);
        return -1;
    }
    i64 m2 = off[n];
    for (int32_t t = 0; t < T; t++) {
        memcpy(start, load, sizeof(i64) * (size_t)n);
        for (int32_t v = 0; v < n; v++) {
            degH[v] = off[v + 1] - off[v];
            inH[v] = 1;
            inF[v] = 0;
        }
        i64 EH = m2 / 2, VH = n;
        i64 it_e = -1, it_v = 1, it_i = 0;
        int32_t j = 0; /* peel counter */
        int improved = 0;
        /* one peel of vertex x: compare, charge, remove */
#define PEEL_ONE(x)                                                                     \
    do {                                                                                \
        int32_t _x = (x);                                                               \
        if (it_e < 0 || (i128)EH * it_v > (i128)it_e * VH) {                            \
            it_e = EH;                                                                  \
            it_v = VH;                                                                  \
            it_i = j;                                                                   \
        }                                                                               \
        if ((i128)EH * best[1] > (i128)best[0] * VH) {                                  \
            best[0] = EH;                                                               \
            best[1] = VH;                                                               \
            best[2] = iter_done + t + 1;                                                \
            best[3] = j;                                                                \
            improved = 1;                                                               \
        }                                                                               \
        load[_x] += degH[_x];                                                           \
        EH -= degH[_x];                                                                 \
        VH -= 1;                                                                        \
        inH[_x] = 0;                                                                    \
        for (int32_t _e = off[_x]; _e < off[_x + 1]; _e++)                              \
            if (inH[adj[_e]]) degH[adj[_e]]--;                                          \
        last_pos[_x] = j;                                                               \
        seq[j] = _x;                                                                    \
        j++;                                                                            \
    } while (0)

        if (variant == ORC_SEQ) {
            while (j < n) {
                int32_t bestv = -1;
                for (int32_t v = 0; v < n; v++) {
                    if (!inH[v]) continue;
                    if (bestv < 0 || start[v] + degH[v] < start[bestv] + degH[bestv]) bestv = v;
                }
                PEEL_ONE(bestv);
            }
        } else if (variant == ORC_PEEL || variant == ORC_PEEL_MONO) {
            i128 dmax = -1;
            while (j < n) {
                i64 mn = -1;
                for (int32_t v = 0; v < n; v++)
                    if (inH[v] && (mn < 0 || start[v] + degH[v] < mn)) mn = start[v] + degH[v];
                i128 lim = (i128)(eps_den + eps_num) * (i128)mn;
                if (variant == ORC_PEEL_MONO) {
                    if (dmax > lim) lim = dmax;
                    dmax = lim;
                }
                for (int32_t v = 0; v < n; v++)
                    inF[v] = inH[v] && (i128)eps_den * (i128)(start[v] + degH[v]) <= lim;
                for (int32_t v = 0; v < n; v++)
                    if (inF[v]) PEEL_ONE(v);
            }
        } else {
            kv* a = (kv*)malloc(sizeof(kv) * (size_t)n);
            if (!a) {
                free(degH); free(start); free(inH); free(seq); free(inF);
                return -1;
            }
            for (int32_t v = 0; v < n; v++) {
                a[v].key = start[v];
                a[v].id = v;
            }
            qsort(a, (size_t)n, sizeof(kv), kv_cmp);
            for (int32_t i = 0; i < n; i++) PEEL_ONE(a[i].id);
            free(a);
        }
#undef PEEL_ONE
        hist[2 * t] = it_e;
        hist[2 * t + 1] = it_v;
        hist_idx[t] = it_i;
        if (improved) memcpy(best_pos, last_pos, sizeof(int32_t) * (size_t)n);
    }
    free(degH); free(start); free(inH); free(seq); free(inF);
    return 0;
}

/*
 * Coreness (Section 2): peel a vertex of minimum current degree, one at a
 * time, until none is left; D is the largest degree any vertex had when it
 * was peeled, and core(v) = D at the moment v is peeled.  The minimum is
 * found with degree buckets (a doubly linked list per degree) so that large
 * graphs finish in O(n + m); which of several minimum-degree vertices goes
 * first does not change any core number.  Returns k_max = max core(v) (0 for
 * a graph without edges), or -1 when out of memory.
 */
int32_t orc_coreness(int32_t n, const int32_t* off, const int32_t* adj, int32_t* core) {
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (off[v + 1] - off[v] > maxd) maxd = off[v + 1] - off[v];
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* head = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd + 1));
    int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* prv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* gone = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!deg || !head || !nxt || !prv || !gone) {
        free(deg); free(head); free(nxt); free(prv); free(gone);
        return -1;
    }
    for (int32_t d = 0; d <= maxd; d++) head[d] = -1;
    for (int32_t v = n - 1; v >= 0; v--) {
        deg[v] = off[v + 1] - off[v];
        prv[v] = -1;
        nxt[v] = head[deg[v]];
        if (head[deg[v]] >= 0) prv[head[deg[v]]] = v;
        head[deg[v]] = v;
    }
    int32_t D = 0, lo = 0;
    for (int32_t step = 0; step < n; step++) {
        while (head[lo] < 0) lo++;  /* lo = current minimum degree */
        const int32_t v = head[lo];
        head[lo] = nxt[v];
        if (nxt[v] >= 0) prv[nxt[v]] = -1;
        gone[v] = 1;
        if (deg[v] > D) D = deg[v];
        core[v] = D;
        for (int32_t e = off[v]; e < off[v + 1]; e++) {
            const int32_t u = adj[e];
            if (gone[u]) continue;
            /* move u from bucket deg[u] to deg[u] - 1 */
            if (prv[u] >= 0) nxt[prv[u]] = nxt[u]; else head[deg[u]] = nxt[u];
            if (nxt[u] >= 0) prv[nxt[u]] = prv[u];
            deg[u]--;
            prv[u] = -1;
            nxt[u] = head[deg[u]];
            if (head[deg[u]] >= 0) prv[head[deg[u]]] = u;
            head[deg[u]] = u;
            if (deg[u] < lo) lo = deg[u];
        }
    }
    free(deg); free(head); free(nxt); free(prv); free(gone);
    return D;
}
