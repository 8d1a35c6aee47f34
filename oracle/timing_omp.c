/*
 * timing_omp.c -- multi-threaded CPU timing build of the Greedy++ iteration.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: nothing on the product
 * path may call, link or load it.  It is not a parity reference either: the
 * plain single-threaded oracle (greedypp_oracle.c) is.  This file exists so
 * that the CPU baseline can be timed on all host cores.  It computes exactly
 * what orc_run computes (the tests require equal outputs on every field), with
 * the same exact-integer rules:
 *   PEEL / PEEL_MONO -- round-synchronous peeling (Section 3.3): per round the
 *       minimum of load + degree over the alive vertices, the frontier of all
 *       alive vertices at or below (1 + eps) times it (PEEL_MONO: at or below
 *       the largest such bound so far), positions by round and ascending id,
 *       and the frontier's effect on its surviving neighbours' degrees applied
 *       at the end of the round;
 *   SORT -- order by (load at the iteration's start, id) (Section 3.2);
 *   then Algorithm 3 (each edge charges its earlier endpoint, suffix sums, the
 *   densest suffix with ties to the smallest index), the load update and the
 *   strict best update of Algorithm 2.
 * Parallel pieces: OpenMP loops with static contiguous chunks (so per-thread
 * counts give id-ordered positions by a prefix over threads), atomic degree
 * decrements and charges, a stable LSD radix sort for SORT.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;
typedef uint64_t u64;
typedef __int128 i128;

enum { T_SEQ = 0, T_PEEL = 1, T_SORT = 2, T_PEEL_MONO = 3 };
#define MAXT 256

static u64 t_mix64(u64 z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* [lo, hi) of thread t's static chunk of k items out of nt threads */
static void chunk(i64 k, int nt, int t, i64* lo, i64* hi) {
    *lo = k * t / nt;
    *hi = k * (t + 1) / nt;
}

/* PEEL ordering on all threads.  alive/next are id-ordered lists; fr holds
 * the round's frontier.  Returns the number of rounds, -1 on no memory. */
static int32_t t_order_peel(int32_t n, const int32_t* off, const int32_t* adj, const i64* load, i64 eps_num,
                            i64 eps_den, int mono, int32_t* pos, int32_t* round, int nt) {
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* alive = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* fr = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !alive || !next || !fr) {
        free(deg); free(alive); free(next); free(fr);
        return -1;
    }
    i64 fcnt[MAXT + 1], scnt[MAXT + 1];
    i64 tmin[MAXT];
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int32_t v = 0; v < n; v++) {
        deg[v] = off[v + 1] - off[v];
        round[v] = -1;
        alive[v] = v;
    }
    int32_t nalive = n, r = 0;
    i64 placed = 0;
    i128 dmax = -1;
    while (nalive > 0) {
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            i64 lo, hi;
            chunk(nalive, nt, t, &lo, &hi);
            i64 m = INT64_MAX;
            for (i64 k = lo; k < hi; k++) {
                const i64 p = load[alive[k]] + deg[alive[k]];
                if (p < m) m = p;
            }
            tmin[t] = m;
        }
        i64 mn = INT64_MAX;
        for (int t = 0; t < nt; t++)
            if (tmin[t] < mn) mn = tmin[t];
        i128 lim = (i128)(eps_den + eps_num) * (i128)mn;
        if (mono) {
            if (dmax > lim) lim = dmax;
            dmax = lim;
        }
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            i64 lo, hi, f = 0, s = 0;
            chunk(nalive, nt, t, &lo, &hi);
            for (i64 k = lo; k < hi; k++) {
                const int32_t v = alive[k];
                if ((i128)eps_den * (i128)(load[v] + deg[v]) <= lim) f++; else s++;
            }
            fcnt[t + 1] = f;
            scnt[t + 1] = s;
#pragma omp barrier
#pragma omp single
            {
                fcnt[0] = 0;
                scnt[0] = 0;
                for (int u = 0; u < nt; u++) {
                    fcnt[u + 1] += fcnt[u];
                    scnt[u + 1] += scnt[u];
                }
            }
            i64 fo = fcnt[t], so = scnt[t];
            for (i64 k = lo; k < hi; k++) {
                const int32_t v = alive[k];
                if ((i128)eps_den * (i128)(load[v] + deg[v]) <= lim) {
                    round[v] = r;
                    pos[v] = (int32_t)(placed + fo);
                    fr[fo++] = v;
                } else {
                    next[so++] = v;
                }
            }
        }
        const i64 nf = fcnt[nt];
        /* delayed effects on the surviving neighbours */
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
        for (i64 k = 0; k < nf; k++) {
            const int32_t v = fr[k];
            for (int32_t e = off[v]; e < off[v + 1]; e++) {
                const int32_t u = adj[e];
                if (round[u] == -1) __atomic_fetch_sub(&deg[u], 1, __ATOMIC_RELAXED);
            }
        }
        placed += nf;
        nalive = (int32_t)scnt[nt];
        int32_t* tmp = alive;
        alive = next;
        next = tmp;
        r++;
    }
    free(deg); free(alive); free(next); free(fr);
    return r;
}

/* SORT ordering: stable LSD radix sort of ids (initially ascending) by load,
 * 8 bits per pass, passes for the bits the largest load uses. */
static int32_t t_order_sort(int32_t n, const i64* load, int32_t* pos, int32_t* round, int nt) {
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* b = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    i64* hist = (i64*)malloc(sizeof(i64) * 256 * (size_t)nt);
    if (!a || !b || !hist) {
        free(a); free(b); free(hist);
        return -1;
    }
    i64 mx = 0;
#pragma omp parallel for num_threads(nt) reduction(max : mx) schedule(static)
    for (int32_t v = 0; v < n; v++) {
        a[v] = v;
        if (load[v] > mx) mx = load[v];
    }
    for (int shift = 0; shift < 64 && (shift == 0 || (mx >> shift) != 0); shift += 8) {
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            i64 lo, hi;
            chunk(n, nt, t, &lo, &hi);
            i64* h = hist + 256 * (size_t)t;
            memset(h, 0, sizeof(i64) * 256);
            for (i64 k = lo; k < hi; k++) h[(load[a[k]] >> shift) & 255]++;
#pragma omp barrier
#pragma omp single
            {
                i64 run = 0;
                for (int d = 0; d < 256; d++)
                    for (int u = 0; u < nt; u++) {
                        const i64 c = hist[256 * (size_t)u + d];
                        hist[256 * (size_t)u + d] = run;
                        run += c;
                    }
            }
            for (i64 k = lo; k < hi; k++) b[h[(load[a[k]] >> shift) & 255]++] = a[k];
        }
        int32_t* tmp = a;
        a = b;
        b = tmp;
    }
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int32_t i = 0; i < n; i++) {
        pos[a[i]] = i;
        round[a[i]] = i;
    }
    free(a); free(b); free(hist);
    return n;
}

/* Algorithm 3 on all threads; same outputs as orc_alg3. */
static void t_alg3(int32_t n, const int32_t* off, const int32_t* adj, const int32_t* pos, i64* A, i64* B, i64* it_e,
                   i64* it_v, i64* it_i, int nt) {
    i64 part[MAXT + 1];
    i64 be_t[MAXT], bv_t[MAXT], bi_t[MAXT];
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int32_t i = 0; i < n; i++) A[i] = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
    for (int32_t u = 0; u < n; u++)
        for (int32_t e = off[u]; e < off[u + 1]; e++) {
            const int32_t v = adj[e];
            if (u < v) __atomic_fetch_add(&A[pos[u] < pos[v] ? pos[u] : pos[v]], 1, __ATOMIC_RELAXED);
        }
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        i64 lo, hi, s = 0;
        chunk(n, nt, t, &lo, &hi);
        for (i64 i = lo; i < hi; i++) s += A[i];
        part[t] = s;
#pragma omp barrier
        i64 run = 0; /* sum of the chunks after this one */
        for (int u = t + 1; u < nt; u++) run += part[u];
        for (i64 i = hi - 1; i >= lo; i--) {
            run += A[i];
            B[i] = run;
        }
        /* best suffix of the chunk, ties to the smallest index */
        i64 be = -1, bv = 1, bi = -1;
        for (i64 i = lo; i < hi; i++) {
            const i64 e = B[i], v = n - i;
            if (bi < 0 || (i128)e * bv > (i128)be * v) {
                be = e;
                bv = v;
                bi = i;
            }
        }
        be_t[t] = be;
        bv_t[t] = bv;
        bi_t[t] = bi;
    }
    i64 be = -1, bv = 1, bi = -1;
    for (int t = 0; t < nt; t++) {
        if (bi_t[t] < 0) continue;
        if (bi < 0 || (i128)be_t[t] * bv > (i128)be * bv_t[t]) {
            be = be_t[t];
            bv = bv_t[t];
            bi = bi_t[t];
        }
    }
    *it_e = be;
    *it_v = bv;
    *it_i = bi;
}

/* Same arguments and outputs as orc_run, plus the thread count (<= 256;
 * 0 = OpenMP's default).  SEQ is not offered (returns -1). */
int orc_run_omp(int32_t n, const int32_t* off, const int32_t* adj, int32_t T, int32_t variant, i64 eps_num,
                i64 eps_den, i64* load, i64* best, int32_t* best_pos, int32_t iter_done, i64* hist, i64* hist_idx,
                u64* digest, int32_t* nrounds, i64* width, int32_t* last_pos, int32_t* last_round, int32_t threads) {
    if (n < 1 || T < 0 || eps_num < 0 || eps_den < 1 || variant == T_SEQ) return -1;
    int nt = threads > 0 ? threads : omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    i64* A = (i64*)malloc(sizeof(i64) * (size_t)n);
    i64* B = (i64*)malloc(sizeof(i64) * (size_t)n);
    if (!A || !B) {
        free(A);
        free(B);
        return -1;
    }
    for (int32_t t = 0; t < T; t++) {
        int32_t rounds;
        if (variant == T_PEEL || variant == T_PEEL_MONO)
            rounds = t_order_peel(n, off, adj, load, eps_num, eps_den, variant == T_PEEL_MONO, last_pos, last_round,
                                  nt);
        else
            rounds = t_order_sort(n, load, last_pos, last_round, nt);
        if (rounds < 0) {
            free(A);
            free(B);
            return -1;
        }
        i64 e, v, i;
        t_alg3(n, off, adj, last_pos, A, B, &e, &v, &i, nt);
        i64 w = 0;
        u64 dg = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(max : w) reduction(+ : dg)
        for (int32_t u = 0; u < n; u++) {
            const i64 inc = A[last_pos[u]];
            load[u] += inc;
            if (inc > w) w = inc;
            dg += t_mix64(((u64)(uint32_t)u << 32) | (u64)(uint32_t)last_round[u]);
        }
        hist[2 * t] = e;
        hist[2 * t + 1] = v;
        hist_idx[t] = i;
        digest[t] = dg;
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
