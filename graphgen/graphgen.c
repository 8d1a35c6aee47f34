/*
 * graphgen.c -- seeded synthetic graph generators (input side only).
 *
 * Holds none of the densest-subgraph method's arithmetic: it only draws
 * undirected simple graphs and emits them as symmetric int32 CSR
 * (offsets[n+1], adj[2m], every row strictly increasing, no self-loops).
 * Both the CPU oracle and the GPU path consume these graphs.
 *
 * Randomness is counter-based: every draw is rnd(seed, stream, index), built
 * from the SplitMix64 output function (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The same (seed, sizes)
 * therefore give the same graph on every x86-64 host, independent of thread
 * count.  Probabilities are exact rationals compared in integer arithmetic.
 *
 * Families (the synthetic stand-ins for the paper's real graphs, whose
 * datasets are not available):
 *   - Erdos-Renyi G(n, m) with exactly m distinct pairs;
 *   - a planted vertex set whose internal pairs appear with probability p;
 *   - R-MAT (recursive quadrant sampling, probabilities a,b,c,d);
 *   - Chung-Lu with power-law weights w_i = C (i+i0)^(-1/(gamma-1)).
 * R-MAT and Chung-Lu ids are relabelled by a seeded permutation so that id
 * order carries no degree information.
 *
 * Memory: a generator returns an opaque handle that owns the CSR; the caller
 * sizes its own arrays from gg_n / gg_nnz, copies with gg_copy, then gg_free.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t u64;
typedef int64_t i64;

enum {
    ST_ER = 1,
    ST_PLANT_SET = 2,
    ST_PLANT_EDGE = 3,
    ST_RMAT = 4,
    ST_PERM = 5,
    ST_CL = 6,
    ST_BLOCK_SET = 7,
    ST_BLOCK_EDGE = 8,
    ST_GNP = 9
};

static inline u64 sm64_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline u64 stream_base(u64 seed, u64 stream) {
    return sm64_mix(seed * 0x9E3779B97F4A7C15ULL + stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL);
}

static inline u64 rnd_at(u64 base, u64 i) { return sm64_mix(base + (i + 1) * 0x9E3779B97F4A7C15ULL); }

static inline u64 rnd(u64 seed, u64 stream, u64 i) { return rnd_at(stream_base(seed, stream), i); }

/* uniform integer in [0, k) by the multiply-shift map of a 64-bit draw */
static inline u64 below(u64 r, u64 k) { return (u64)(((unsigned __int128)r * k) >> 64); }

/* ---------------------------------------------------------------- handle */
typedef struct {
    i64 n;
    i64 nnz;
    int32_t* offsets;
    int32_t* adj;
    char err[160];
} gg_graph;

i64 gg_n(const gg_graph* g) { return g ? g->n : -1; }
i64 gg_nnz(const gg_graph* g) { return g ? g->nnz : -1; }
const char* gg_error(const gg_graph* g) { return g ? g->err : "null handle"; }

void gg_free(gg_graph* g) {
    if (!g) return;
    free(g->offsets);
    free(g->adj);
    free(g);
}

int gg_copy(const gg_graph* g, int32_t* offsets, int32_t* adj) {
    if (!g || !g->offsets) return -1;
    memcpy(offsets, g->offsets, (size_t)(g->n + 1) * sizeof(int32_t));
    if (g->nnz) memcpy(adj, g->adj, (size_t)g->nnz * sizeof(int32_t));
    return 0;
}

/* ------------------------------------------------- sort / unique / CSR build */
/* LSD radix sort of 64-bit keys, 16-bit digits; passes whose digit is constant
 * over all keys are skipped. */
static int radix_sort_u64(u64* a, i64 cnt, int key_bits) {
    if (cnt <= 1) return 0;
    u64* tmp = (u64*)malloc((size_t)cnt * sizeof(u64));
    if (!tmp) return -1;
    i64* hist = (i64*)malloc(65536 * sizeof(i64));
    if (!hist) { free(tmp); return -1; }
    u64* src = a;
    u64* dst = tmp;
    for (int shift = 0; shift < key_bits; shift += 16) {
        memset(hist, 0, 65536 * sizeof(i64));
        for (i64 i = 0; i < cnt; i++) hist[(src[i] >> shift) & 0xFFFF]++;
        int single = 0;
        for (int d = 0; d < 65536; d++)
            if (hist[d] == cnt) single = 1;
        if (single) continue;
        i64 run = 0;
        for (int d = 0; d < 65536; d++) {
            i64 c = hist[d];
            hist[d] = run;
            run += c;
        }
        for (i64 i = 0; i < cnt; i++) dst[hist[(src[i] >> shift) & 0xFFFF]++] = src[i];
        u64* t = src;
        src = dst;
        dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)cnt * sizeof(u64));
    free(tmp);
    free(hist);
    return 0;
}

/* keys hold (min << 32) | max of undirected pairs, self-loops already removed.
 * Sorts, drops duplicates and writes a symmetric CSR into g. */
static int build_csr(gg_graph* g, i64 n, u64* keys, i64 cnt) {
    int bits = 64;
    if (radix_sort_u64(keys, cnt, bits) != 0) {
        strcpy(g->err, "out of memory in sort");
        return -1;
    }
    i64 m = 0;
    for (i64 i = 0; i < cnt; i++)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    if (2 * m > (i64)INT32_MAX) {
        strcpy(g->err, "graph too large for int32 CSR");
        return -1;
    }
    g->n = n;
    g->nnz = 2 * m;
    g->offsets = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    g->adj = (int32_t*)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    if (!g->offsets || !g->adj) {
        strcpy(g->err, "out of memory in CSR build");
        return -1;
    }
    for (i64 i = 0; i < m; i++) {
        g->offsets[(keys[i] >> 32) + 1]++;
        g->offsets[(keys[i] & 0xFFFFFFFFULL) + 1]++;
    }
    for (i64 v = 0; v < n; v++) g->offsets[v + 1] += g->offsets[v];
    int32_t* fill = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!fill) {
        strcpy(g->err, "out of memory in CSR build");
        return -1;
    }
    memcpy(fill, g->offsets, (size_t)n * sizeof(int32_t));
    /* keys are sorted by (a, b) with a < b: row a receives b in ascending b,
     * and row b receives a in ascending a, after every entry c < a of row a
     * that arrived earlier -- so every row comes out strictly increasing. */
    for (i64 i = 0; i < m; i++) {
        u64 a = keys[i] >> 32, b = keys[i] & 0xFFFFFFFFULL;
        g->adj[fill[a]++] = (int32_t)b;
        g->adj[fill[b]++] = (int32_t)a;
    }
    free(fill);
    return 0;
}

static inline u64 pair_key(u64 u, u64 v) { return u < v ? (u << 32) | v : (v << 32) | u; }

static gg_graph* new_graph(void) { return (gg_graph*)calloc(1, sizeof(gg_graph)); }

/* seeded uniform permutation of [0, n) by Fisher-Yates */
static int32_t* make_perm(u64 seed, i64 n) {
    int32_t* p = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!p) return NULL;
    for (i64 i = 0; i < n; i++) p[i] = (int32_t)i;
    for (i64 i = n - 1; i > 0; i--) {
        i64 j = (i64)below(rnd(seed, ST_PERM, (u64)i), (u64)(i + 1));
        int32_t t = p[i];
        p[i] = p[j];
        p[j] = t;
    }
    return p;
}

/* ------------------------------------------------------------- hash set */
typedef struct {
    u64* slot;
    u64 mask;
    i64 count;
} hset;

static int hset_init(hset* h, i64 expect) {
    u64 cap = 16;
    while (cap < (u64)(expect * 2 + 16)) cap <<= 1;
    h->slot = (u64*)malloc(cap * sizeof(u64));
    if (!h->slot) return -1;
    memset(h->slot, 0xFF, cap * sizeof(u64));
    h->mask = cap - 1;
    h->count = 0;
    return 0;
}

/* returns 1 if inserted, 0 if present (keys never equal UINT64_MAX) */
static int hset_insert(hset* h, u64 key) {
    u64 i = sm64_mix(key) & h->mask;
    while (h->slot[i] != UINT64_MAX) {
        if (h->slot[i] == key) return 0;
        i = (i + 1) & h->mask;
    }
    h->slot[i] = key;
    h->count++;
    return 1;
}

/* ---------------------------------------------------------- generators */

/* Erdos-Renyi G(n, m) plus a planted set.
 * ER part: draw pairs (u, v), u != v, in counter order, keep the first m distinct
 * ones.  Planted part (k > 0): the first k entries of a seeded permutation form
 * the set; each of its k(k-1)/2 internal pairs is added with probability
 * p_num/p_den (added on top of the m ER edges; duplicates merge). */
gg_graph* gg_er_planted(u64 seed, i64 n, i64 m, i64 k, i64 p_num, i64 p_den) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (n < 1 || n > INT32_MAX || m < 0 || k < 0 || k > n || p_den <= 0 || p_num < 0 || p_num > p_den) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    if (m > n * (n - 1) / 2) {
        strcpy(g->err, "m exceeds the number of pairs");
        return g;
    }
    i64 cap = m + k * (k - 1) / 2 + 1;
    u64* keys = (u64*)malloc((size_t)cap * sizeof(u64));
    hset h;
    if (!keys || hset_init(&h, m) != 0) {
        free(keys);
        strcpy(g->err, "out of memory");
        return g;
    }
    i64 cnt = 0;
    for (u64 i = 0; cnt < m; i++) {
        u64 r = rnd(seed, ST_ER, i);
        u64 u = below(r, (u64)n);
        u64 v = below(rnd(seed, ST_ER, i ^ (1ULL << 62)), (u64)n);
        if (u == v) continue;
        u64 key = pair_key(u, v);
        if (hset_insert(&h, key)) keys[cnt++] = key;
    }
    free(h.slot);
    if (k > 1) {
        int32_t* perm = make_perm(seed ^ 0xA5A5A5A5ULL, n);
        if (!perm) {
            free(keys);
            strcpy(g->err, "out of memory");
            return g;
        }
        u64 idx = 0;
        for (i64 a = 0; a < k; a++)
            for (i64 b = a + 1; b < k; b++, idx++) {
                u64 r = rnd(seed, ST_PLANT_EDGE, idx);
                /* accept with probability p_num / p_den exactly */
                if (below(r, (u64)p_den) < (u64)p_num) keys[cnt++] = pair_key((u64)perm[a], (u64)perm[b]);
            }
        free(perm);
    }
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* G(n, p) over all pairs (tiny test graphs): pair (a<b) present iff its draw
 * falls below p_num/p_den. */
gg_graph* gg_gnp(u64 seed, i64 n, i64 p_num, i64 p_den) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (n < 1 || n > 100000 || p_den <= 0 || p_num < 0 || p_num > p_den) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    i64 cap = n * (n - 1) / 2 + 1;
    u64* keys = (u64*)malloc((size_t)cap * sizeof(u64));
    if (!keys) {
        strcpy(g->err, "out of memory");
        return g;
    }
    i64 cnt = 0;
    u64 idx = 0;
    for (i64 a = 0; a < n; a++)
        for (i64 b = a + 1; b < n; b++, idx++)
            if (below(rnd(seed, ST_GNP, idx), (u64)p_den) < (u64)p_num) keys[cnt++] = pair_key((u64)a, (u64)b);
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* CSR from an explicit edge list (u[i], v[i]); self-loops dropped, duplicates
 * merged.  For hand-made test graphs. */
gg_graph* gg_from_edges(i64 n, const int32_t* u, const int32_t* v, i64 count) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (n < 1 || n > INT32_MAX || count < 0) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    u64* keys = (u64*)malloc((size_t)(count > 0 ? count : 1) * sizeof(u64));
    if (!keys) {
        strcpy(g->err, "out of memory");
        return g;
    }
    i64 cnt = 0;
    for (i64 i = 0; i < count; i++) {
        if (u[i] < 0 || v[i] < 0 || u[i] >= n || v[i] >= n) {
            free(keys);
            strcpy(g->err, "endpoint out of range");
            return g;
        }
        if (u[i] != v[i]) keys[cnt++] = pair_key((u64)u[i], (u64)v[i]);
    }
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* R-MAT: `samples` draws, each descends `scale` levels choosing quadrant
 * (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1) w.p. d = 1-a-b-c, with a,b,c
 * given in hundredths.  Endpoints >= n are redrawn from the next counter index
 * (n < 2^scale only for the batched mix).  Self-loops dropped, pairs
 * symmetrised and deduplicated, ids relabelled by a seeded permutation when
 * relabel != 0. */
gg_graph* gg_rmat(u64 seed, int scale, i64 n, i64 samples, int a100, int b100, int c100, int relabel) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (scale < 1 || scale > 30 || n < 1 || n > (1LL << scale) || samples < 0 || a100 < 0 || b100 < 0 || c100 < 0 ||
        a100 + b100 + c100 > 100) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    u64* keys = (u64*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(u64));
    if (!keys) {
        strcpy(g->err, "out of memory");
        return g;
    }
    const u64 ta = (u64)a100, tb = (u64)(a100 + b100), tc = (u64)(a100 + b100 + c100);
    const u64 base = stream_base(seed, ST_RMAT);
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < samples; s++) {
        u64 key = UINT64_MAX;
        for (u64 attempt = 0; attempt < 64; attempt++) {
            u64 u = 0, v = 0;
            u64 ctr = ((u64)s << 6 | attempt) * 32;
            for (int lvl = 0; lvl < scale; lvl++) {
                /* one draw per level; quadrant by its value below 100 */
                u64 q = below(rnd_at(base, ctr + (u64)lvl), 100);
                u64 bu = (q >= tb), bv = (q >= ta && q < tb) || (q >= tc);
                u = (u << 1) | bu;
                v = (v << 1) | bv;
            }
            if (u >= (u64)n || v >= (u64)n) continue;
            key = (u == v) ? UINT64_MAX - 1 : pair_key(u, v);
            break;
        }
        keys[s] = key;
    }
    int32_t* perm = relabel ? make_perm(seed ^ 0x5EED5EEDULL, n) : NULL;
    i64 cnt = 0;
    for (i64 s = 0; s < samples; s++) {
        if (keys[s] >= UINT64_MAX - 1) continue;
        u64 u = keys[s] >> 32, v = keys[s] & 0xFFFFFFFFULL;
        if (perm) {
            u = (u64)perm[u];
            v = (u64)perm[v];
        }
        keys[cnt++] = pair_key(u, v);
    }
    free(perm);
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* Chung-Lu with power-law weights.  w_i = C (i + i0)^(-1/(gamma-1)) for
 * i = 0..n-1, with (C, i0) chosen so that w_0 = max_deg and the mean weight is
 * mean_deg (i0 by bisection on the integral approximation of the sum).
 * n*mean_deg/2 endpoint pairs are drawn with both endpoints proportional to w
 * (Walker alias table over integer-scaled weights), loops and duplicates
 * dropped, ids relabelled by a seeded permutation. */
gg_graph* gg_chunglu(u64 seed, i64 n, double gamma, double mean_deg, double max_deg, int relabel) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (n < 2 || n > INT32_MAX || gamma <= 2.0 || mean_deg <= 0 || max_deg < mean_deg) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    const double a = 1.0 / (gamma - 1.0);
    /* mean(i0) = max_deg * i0^a / n * S(i0), S = sum_{i<n} (i+i0)^-a
     * ~ ((n+i0)^(1-a) - i0^(1-a)) / (1-a) + (i0^-a + (n-1+i0)^-a)/2 */
    double lo = 1e-9, hi = (double)n * 1e6;
    for (int it = 0; it < 300; it++) {
        double i0 = sqrt(lo * hi);
        double S = (pow((double)n + i0, 1 - a) - pow(i0, 1 - a)) / (1 - a) + 0.5 * (pow(i0, -a) + pow(n - 1 + i0, -a));
        double mean = max_deg * pow(i0, a) / (double)n * S;
        if (mean > mean_deg) hi = i0; else lo = i0;
    }
    const double i0 = sqrt(lo * hi);
    const double C = max_deg * pow(i0, a);
    /* integer weights, scaled so the total stays below 2^62 */
    double* wd = (double*)malloc((size_t)n * sizeof(double));
    u64* w = (u64*)malloc((size_t)n * sizeof(u64));
    u64* prob = (u64*)malloc((size_t)n * sizeof(u64));
    int32_t* alias = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* small = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* large = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    i64 samples = (i64)((double)n * mean_deg / 2.0);
    u64* keys = (u64*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(u64));
    if (!wd || !w || !prob || !alias || !small || !large || !keys) {
        free(wd); free(w); free(prob); free(alias); free(small); free(large); free(keys);
        strcpy(g->err, "out of memory");
        return g;
    }
    double tot = 0;
    for (i64 i = 0; i < n; i++) {
        wd[i] = C * pow((double)i + i0, -a);
        tot += wd[i];
    }
    const double scale = ldexp(1.0, 61) / tot;
    u64 W = 0;
    for (i64 i = 0; i < n; i++) {
        w[i] = (u64)(wd[i] * scale) + 1;
        W += w[i];
    }
    free(wd);
    /* Walker/Vose alias table in exact integers: column i keeps itself with
     * probability prob[i]/W, else takes alias[i].  Column mass is W/n in
     * units where every weight is multiplied by n. */
    i64 ns = 0, nl = 0;
    for (i64 i = 0; i < n; i++) {
        /* scaled weight n*w[i] compared with W */
        unsigned __int128 sw = (unsigned __int128)w[i] * (u64)n;
        if (sw < W) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
    }
    /* residual masses, in units of 1/n of a weight */
    unsigned __int128* res = (unsigned __int128*)malloc((size_t)n * sizeof(unsigned __int128));
    if (!res) {
        free(w); free(prob); free(alias); free(small); free(large); free(keys);
        strcpy(g->err, "out of memory");
        return g;
    }
    for (i64 i = 0; i < n; i++) res[i] = (unsigned __int128)w[i] * (u64)n;
    while (ns > 0 && nl > 0) {
        int32_t s = small[--ns];
        int32_t l = large[nl - 1];
        prob[s] = (u64)res[s]; /* < W */
        alias[s] = l;
        res[l] -= (unsigned __int128)W - res[s];
        if (res[l] < W) {
            nl--;
            small[ns++] = l;
        }
    }
    while (nl > 0) { int32_t l = large[--nl]; prob[l] = W; alias[l] = l; }
    while (ns > 0) { int32_t s = small[--ns]; prob[s] = W; alias[s] = s; }
    free(res);
    free(small);
    free(large);
    free(w);
    const u64 cbase = stream_base(seed, ST_CL);
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < samples; s++) {
        u64 e[2];
        for (int k = 0; k < 2; k++) {
            u64 col = below(rnd_at(cbase, 4 * (u64)s + 2 * (u64)k), (u64)n);
            u64 r = below(rnd_at(cbase, 4 * (u64)s + 2 * (u64)k + 1), W);
            e[k] = r < prob[col] ? col : (u64)alias[col];
        }
        keys[s] = (e[0] == e[1]) ? UINT64_MAX : pair_key(e[0], e[1]);
    }
    free(prob);
    free(alias);
    int32_t* perm = relabel ? make_perm(seed ^ 0xC1C1C1C1ULL, n) : NULL;
    i64 cnt = 0;
    for (i64 s = 0; s < samples; s++) {
        if (keys[s] == UINT64_MAX) continue;
        u64 u = keys[s] >> 32, v = keys[s] & 0xFFFFFFFFULL;
        if (perm) {
            u = (u64)perm[u];
            v = (u64)perm[v];
        }
        keys[cnt++] = pair_key(u, v);
    }
    free(perm);
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* ER G(n, M samples, deduplicated) plus a dense block on a seeded subset of
 * `block` vertices with internal pair probability p_num/p_den. */
gg_graph* gg_er_block(u64 seed, i64 n, i64 samples, i64 block, i64 p_num, i64 p_den) {
    gg_graph* g = new_graph();
    if (!g) return NULL;
    if (n < 2 || n > INT32_MAX || samples < 0 || block < 0 || block > n || p_den <= 0 || p_num < 0 || p_num > p_den) {
        strcpy(g->err, "bad parameters");
        return g;
    }
    /* expected block pairs plus slack; counted exactly below */
    i64 bp = 0;
    u64 idx = 0;
    for (i64 a = 0; a < block; a++)
        for (i64 b = a + 1; b < block; b++, idx++)
            if (below(rnd(seed, ST_BLOCK_EDGE, idx), (u64)p_den) < (u64)p_num) bp++;
    u64* keys = (u64*)malloc((size_t)(samples + bp + 1) * sizeof(u64));
    if (!keys) {
        strcpy(g->err, "out of memory");
        return g;
    }
    i64 cnt = 0;
    for (i64 s = 0; s < samples; s++) {
        u64 u = below(rnd(seed, ST_ER, 2 * (u64)s), (u64)n);
        u64 v = below(rnd(seed, ST_ER, 2 * (u64)s + 1), (u64)n);
        if (u != v) keys[cnt++] = pair_key(u, v);
    }
    if (block > 1) {
        int32_t* perm = make_perm(seed ^ 0xB10CB10CULL, n);
        if (!perm) {
            free(keys);
            strcpy(g->err, "out of memory");
            return g;
        }
        idx = 0;
        for (i64 a = 0; a < block; a++)
            for (i64 b = a + 1; b < block; b++, idx++)
                if (below(rnd(seed, ST_BLOCK_EDGE, idx), (u64)p_den) < (u64)p_num)
                    keys[cnt++] = pair_key((u64)perm[a], (u64)perm[b]);
        free(perm);
    }
    build_csr(g, n, keys, cnt);
    free(keys);
    return g;
}

/* exposed for the batched-mix sampler: the same counter-based draw */
u64 gg_rnd(u64 seed, u64 stream, u64 i) { return rnd(seed, stream, i); }
