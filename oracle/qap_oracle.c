/*
 * qap_oracle.c -- plain, slow CPU oracle for the pairwise-exchange QAP heuristics
 * of Novoa & Qasem, "GPU-accelerated Parallel Solutions to the Quadratic
 * Assignment Problem" (arXiv 2307.11248).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  The product library never
 * links, includes or calls it, and it shares no code with the HIP path.
 *
 * Conventions (Sec. 2.1 of the paper, restated 0-based):
 *   F[k*n + l]  flow between units k and l        (row-major n x n, int32)
 *   D[i*n + j]  distance between locations i, j  (row-major n x n, int32)
 *   p[i]        unit stored in location i          (a permutation of 0..n-1)
 * A move (r, s) with r < s exchanges the contents of locations r and s.
 * Moves are numbered in packed upper-triangle order
 *   idx(r, s) = r*n - r*(r+1)/2 + (s - r - 1),
 * which is lexicographic order of (r, s); ties are broken by lowest idx.
 *
 * All arithmetic is exact integer arithmetic in int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

static int64_t pidx(int n, int r, int s) {
    return (int64_t)r * n - (int64_t)r * (r + 1) / 2 + (s - r - 1);
}

/* Cost of a permutation, Eq. (1): z = sum_i sum_j f[p_i][p_j] * d[i][j]. */
ORC_EXPORT int64_t orc_cost(int n, const int32_t *F, const int32_t *D, const int32_t *p) {
    int64_t z = 0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            z += (int64_t)F[(int64_t)p[i] * n + p[j]] * D[(int64_t)i * n + j];
    return z;
}

/*
 * Change in cost when the contents of locations r and s are exchanged: the
 * Burkard-Rendl formula, Eq. (2), for asymmetric F and D, plus the term
 * (d_ss - d_rr)(f_{p_r p_r} - f_{p_s p_s}) that the printed equation leaves
 * out; that term is zero whenever D has a zero diagonal.
 */
ORC_EXPORT int64_t orc_delta(int n, const int32_t *F, const int32_t *D, const int32_t *p,
                             int r, int s) {
#define f(a, b) ((int64_t)F[(int64_t)(a) * n + (b)])
#define d(a, b) ((int64_t)D[(int64_t)(a) * n + (b)])
    int pr = p[r], ps = p[s];
    int64_t delta = (d(s, s) - d(r, r)) * (f(pr, pr) - f(ps, ps))
                  + (d(s, r) - d(r, s)) * (f(pr, ps) - f(ps, pr));
    for (int k = 0; k < n; k++) {
        if (k == r || k == s) continue;
        int pk = p[k];
        delta += (d(s, k) - d(r, k)) * (f(pr, pk) - f(ps, pk))
               + (d(k, s) - d(k, r)) * (f(pk, pr) - f(pk, ps));
    }
    return delta;
#undef f
#undef d
}

/* The whole pairwise-exchange neighbourhood (Sec. 4.1), one Eq. (2) per move,
 * written in packed order: out[idx(r,s)] = delta(p, r, s). */
ORC_EXPORT void orc_delta_table(int n, const int32_t *F, const int32_t *D, const int32_t *p,
                                int64_t *out) {
    for (int r = 0; r < n; r++)
        for (int s = r + 1; s < n; s++)
            out[pidx(n, r, s)] = orc_delta(n, F, D, p, r, s);
}

/*
 * The whole neighbourhood in contraction form: with G[a][b] = F[p_a][p_b] and
 * T = G.D^T + G^T.D (two n x n x n products),
 *   delta(i, j) = T_ij + T_ji - T_ii - T_jj + c_ij,
 * where c_ij gathers the k = i and k = j terms of Eq. (2) (with its diagonal
 * term) that the sums over all k count differently:
 *   c_ij = -(D_ji - D_ii)(G_ii - G_ji) - (D_jj - D_ij)(G_ij - G_jj)
 *          -(D_ij - D_ii)(G_ii - G_ij) - (D_jj - D_ji)(G_ji - G_jj)
 *          +(D_ji - D_ij)(G_ij - G_ji) + (D_jj - D_ii)(G_ii - G_jj).
 * Written out with plain loops; it must equal orc_delta_table exactly.
 */
ORC_EXPORT void orc_delta_table_contraction(int n, const int32_t *F, const int32_t *D, const int32_t *p,
                                            int64_t *out) {
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * n);
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * n);
    if (!G || !T) {
        free(G);
        free(T);
        return;
    }
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) G[(size_t)a * n + b] = F[(size_t)p[a] * n + p[b]];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int64_t t = 0;
            for (int k = 0; k < n; k++)
                t += G[(size_t)i * n + k] * D[(size_t)j * n + k]      /* (G D^T)_ij */
                   + G[(size_t)k * n + i] * D[(size_t)k * n + j];     /* (G^T D)_ij */
            T[(size_t)i * n + j] = t;
        }
#define GG(a, b) G[(size_t)(a) * n + (b)]
#define DD(a, b) ((int64_t)D[(size_t)(a) * n + (b)])
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            const int64_t c = -(DD(j, i) - DD(i, i)) * (GG(i, i) - GG(j, i))
                              - (DD(j, j) - DD(i, j)) * (GG(i, j) - GG(j, j))
                              - (DD(i, j) - DD(i, i)) * (GG(i, i) - GG(i, j))
                              - (DD(j, j) - DD(j, i)) * (GG(j, i) - GG(j, j))
                              + (DD(j, i) - DD(i, j)) * (GG(i, j) - GG(j, i))
                              + (DD(j, j) - DD(i, i)) * (GG(i, i) - GG(j, j));
            out[pidx(n, i, j)] = T[(size_t)i * n + j] + T[(size_t)j * n + i] - T[(size_t)i * n + i] -
                                 T[(size_t)j * n + j] + c;
        }
#undef GG
#undef DD
    free(G);
    free(T);
}

/*
 * Incremental neighbourhood update after the move (r, s) has been applied
 * (Taillard 1991, the reference the paper follows for its elementary tabu
 * search).  `p_before` is the permutation BEFORE the move; `tab` holds the
 * deltas of p_before in packed order and is overwritten with those of the new
 * permutation.
 *   For pairs (u, v) disjoint from {r, s}, only the k = r and k = s terms of
 *   Eq. (2) change, which gives
 *     delta'(u,v) = delta(u,v) + (A_u - A_v)(B_u - B_v) + (C_u - C_v)(E_u - E_v)
 *   with A_u = d_ur - d_us, C_u = d_ru - d_su,
 *        B_u = f[p_u][p_r] - f[p_u][p_s], E_u = f[p_r][p_u] - f[p_s][p_u].
 *   The pair (r, s) itself is undone by repeating it: delta'(r,s) = -delta(r,s).
 *   Every other pair that touches r or s is recomputed with Eq. (2) under the
 *   new permutation.
 */
ORC_EXPORT void orc_delta_update(int n, const int32_t *F, const int32_t *D,
                                 const int32_t *p_before, int r, int s, int64_t *tab) {
#define f(a, b) ((int64_t)F[(int64_t)(a) * n + (b)])
#define d(a, b) ((int64_t)D[(int64_t)(a) * n + (b)])
    if (r > s) { int t = r; r = s; s = t; }
    int64_t *A = malloc(sizeof(int64_t) * n), *B = malloc(sizeof(int64_t) * n);
    int64_t *C = malloc(sizeof(int64_t) * n), *E = malloc(sizeof(int64_t) * n);
    int32_t *q = malloc(sizeof(int32_t) * n);
    int pr = p_before[r], ps = p_before[s];
    for (int u = 0; u < n; u++) {
        int pu = p_before[u];
        A[u] = d(u, r) - d(u, s);
        C[u] = d(r, u) - d(s, u);
        B[u] = f(pu, pr) - f(pu, ps);
        E[u] = f(pr, pu) - f(ps, pu);
    }
    memcpy(q, p_before, sizeof(int32_t) * n);
    q[r] = ps; q[s] = pr;
    for (int u = 0; u < n; u++) {
        for (int v = u + 1; v < n; v++) {
            int64_t i = pidx(n, u, v);
            if (u == r && v == s)
                tab[i] = -tab[i];
            else if (u == r || u == s || v == r || v == s)
                tab[i] = orc_delta(n, F, D, q, u, v);
            else
                tab[i] += (A[u] - A[v]) * (B[u] - B[v]) + (C[u] - C[v]) * (E[u] - E[v]);
        }
    }
    free(A); free(B); free(C); free(E); free(q);
#undef f
#undef d
}

/*
 * Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
 * published definition: ten rounds of two 64x64->128-bit multiplications
 * with a Weyl-sequence key schedule.
 */
ORC_EXPORT void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                                  uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 m0 = (unsigned __int128)M0 * c0;
        unsigned __int128 m1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(m0 >> 64), lo0 = (uint64_t)m0;
        uint64_t hi1 = (uint64_t)(m1 >> 64), lo1 = (uint64_t)m1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Dynamic tabu tenure (Sec. 4.3): one integer drawn uniformly from [lo, hi]
 * each time a move is made tabu.  The draw for iteration `it` of start
 * `start` under `seed` is the first output word x of Philox4x64-10 with
 * key (seed, 0) and counter (it, start, 0, 0); it is mapped to the range by
 * the multiply-shift method on its upper 32 bits:
 *   t = lo + ((x >> 32) * (hi - lo + 1)) >> 32.
 */
ORC_EXPORT int32_t orc_tenure(uint64_t seed, uint64_t it, uint64_t start, int32_t lo, int32_t hi) {
    uint64_t ctr[4] = {it, start, 0, 0}, key[2] = {seed, 0}, x[4];
    orc_philox4x64_10(ctr, key, x);
    uint64_t span = (uint64_t)((int64_t)hi - lo + 1);
    return lo + (int32_t)(((x[0] >> 32) * span) >> 32);
}

typedef struct { int64_t delta; int64_t idx; } cand_t;

static int cand_cmp(const void *a, const void *b) {
    const cand_t *x = a, *y = b;
    if (x->delta != y->delta) return x->delta < y->delta ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static void pair_of(int n, int64_t idx, int *r, int *s) {
    int u = 0;
    while (idx >= n - 1 - u) { idx -= n - 1 - u; u++; }
    *r = u; *s = u + 1 + (int)idx;
}

/*
 * 2opt (Sec. 4.1): evaluate the whole pairwise-exchange neighbourhood, move to
 * its best member, repeat.  Read as best improvement: the search stops at the
 * first permutation with no improving exchange (a local optimum), or after
 * max_iters moves when max_iters > 0.  Ties go to the lowest packed index.
 *   mode 0: every neighbourhood is evaluated afresh with Eq. (2);
 *   mode 1: the neighbourhood is kept up to date with orc_delta_update.
 * On return p holds the final permutation (the best one: the cost strictly
 * decreases), *cost its cost and *steps the number of moves made.  If trace
 * is not NULL, move t writes (r, s, delta, cost after) to trace[4t..4t+3] for
 * t < trace_cap.  Returns 0, or -1 if memory ran out.
 */
ORC_EXPORT int orc_2opt(int n, const int32_t *F, const int32_t *D, int32_t *p,
                        int32_t max_iters, int mode, int64_t *cost, int32_t *steps,
                        int64_t *trace, int32_t trace_cap) {
    int64_t m = (int64_t)n * (n - 1) / 2;
    int64_t *tab = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    if (!tab) return -1;
    int64_t z = orc_cost(n, F, D, p);
    int32_t t = 0;
    if (m > 0) orc_delta_table(n, F, D, p, tab);
    while (m > 0 && (max_iters <= 0 || t < max_iters)) {
        if (mode == 0 && t > 0) orc_delta_table(n, F, D, p, tab);
        int64_t best = 0;
        for (int64_t i = 1; i < m; i++)
            if (tab[i] < tab[best]) best = i;
        if (tab[best] >= 0) break;
        int r, s;
        pair_of(n, best, &r, &s);
        int64_t dz = tab[best];
        if (mode == 1) orc_delta_update(n, F, D, p, r, s, tab);
        int32_t tmp = p[r]; p[r] = p[s]; p[s] = tmp;
        z += dz;
        if (trace && t < trace_cap) {
            trace[4 * t] = r; trace[4 * t + 1] = s; trace[4 * t + 2] = dz; trace[4 * t + 3] = z;
        }
        t++;
    }
    free(tab);
    *cost = z;
    if (steps) *steps = t;
    return 0;
}

/*
 * Elementary tabu search with recency memory (Secs. 4.3 and 4.4).
 *   Iterations are numbered it = 1 .. iters.
 *   Tabuarr holds, for each move, the first iteration at which it is free
 *   again: the move is tabu at iteration it iff Tabuarr > it.  It starts at 0.
 *   Aspiration: a tabu move is allowed if it reaches a cost strictly lower
 *   than the best cost found so far (the best before this move).
 *   Among the allowed moves the one with the lowest delta is taken, even if
 *   it worsens the cost; ties go to the lowest packed index.
 *   The current solution becomes the best one when its cost is strictly lower.
 *   After the move (r, s) of iteration it, Tabuarr(r, s) = it + t with t the
 *   tenure drawn by orc_tenure(seed, it, start, lo, hi).
 *   If no move is allowed the search stops early; *iters_done counts the
 *   moves that were made.
 *   mode 0 follows the paper's description literally: each iteration all
 *   deltas are recomputed with Eq. (2), the moves are ranked by (delta, idx)
 *   and the ranking is walked until an allowed move is found.
 *   mode 1 keeps the deltas with orc_delta_update and takes the minimum over
 *   the allowed moves by a linear scan.
 * The frequency counters of the lower triangle of Tabuarr affect no decision
 * and are not kept.  best_perm receives the best permutation, *best_cost its
 * cost.  Trace rows are (r, s, delta, cost after) as in orc_2opt.
 * Returns 0, or -1 if memory ran out.
 */
ORC_EXPORT int orc_tabu(int n, const int32_t *F, const int32_t *D, const int32_t *p0,
                        int32_t iters, int32_t lo, int32_t hi, uint64_t seed, uint64_t start,
                        int mode, int32_t *best_perm, int64_t *best_cost, int32_t *iters_done,
                        int64_t *trace, int32_t trace_cap) {
    int64_t m = (int64_t)n * (n - 1) / 2;
    int64_t *tab = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    int64_t *until = calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    cand_t *cand = malloc(sizeof(cand_t) * (m > 0 ? m : 1));
    int32_t *p = malloc(sizeof(int32_t) * n);
    if (!tab || !until || !cand || !p) { free(tab); free(until); free(cand); free(p); return -1; }
    memcpy(p, p0, sizeof(int32_t) * n);
    memcpy(best_perm, p0, sizeof(int32_t) * n);
    int64_t cur = orc_cost(n, F, D, p), best = cur;
    int32_t done = 0;
    if (m > 0) orc_delta_table(n, F, D, p, tab);
    for (int32_t it = 1; it <= iters && m > 0; it++) {
        int64_t pick = -1;
        if (mode == 0) {
            if (it > 1) orc_delta_table(n, F, D, p, tab);
            for (int64_t i = 0; i < m; i++) { cand[i].delta = tab[i]; cand[i].idx = i; }
            qsort(cand, (size_t)m, sizeof(cand_t), cand_cmp);
            for (int64_t c = 0; c < m; c++) {
                int64_t i = cand[c].idx;
                if (until[i] <= it || cur + tab[i] < best) { pick = i; break; }
            }
        } else {
            for (int64_t i = 0; i < m; i++) {
                if (!(until[i] <= it || cur + tab[i] < best)) continue;
                if (pick < 0 || tab[i] < tab[pick]) pick = i;
            }
        }
        if (pick < 0) break;
        int r, s;
        pair_of(n, pick, &r, &s);
        int64_t dz = tab[pick];
        if (mode == 1) orc_delta_update(n, F, D, p, r, s, tab);
        int32_t tmp = p[r]; p[r] = p[s]; p[s] = tmp;
        cur += dz;
        if (cur < best) { best = cur; memcpy(best_perm, p, sizeof(int32_t) * n); }
        until[pick] = (int64_t)it + orc_tenure(seed, (uint64_t)it, start, lo, hi);
        if (trace && done < trace_cap) {
            trace[4 * done] = r; trace[4 * done + 1] = s;
            trace[4 * done + 2] = dz; trace[4 * done + 3] = cur;
        }
        done = it;
    }
    *best_cost = best;
    if (iters_done) *iters_done = done;
    free(tab); free(until); free(cand); free(p);
    return 0;
}

/*
 * Tabu search that keeps the frequency memory of Sec. 4.3 -- freq[i], the number of
 * moves made with packed index i (the paper's lower triangle of Tabuarr) -- may use it
 * to diversify, and may use a unit-based tabu attribute instead of the pair one.  The paper records the counts but diversifies only through the
 * dynamic tenure, leaving a frequency-based rule to future work (Sec. 7); the rule here
 * is this build's reading of that intent:
 *   last = the iteration at which the best cost last improved (0 before any).
 *   div > 0 and it - last > div: a diversification move.  Among the moves that are not
 *     tabu (Tabuarr <= it; no aspiration) the one exchanged least often so far is taken,
 *     ties to the lowest packed index, whatever its delta; afterwards last = it.  If
 *     every move is tabu the iteration follows the ordinary rule.
 *   Otherwise (and always when div = 0) the ordinary rule of orc_tabu.
 * attr selects what is tabu:
 *   0: the pair of locations, as in orc_tabu (Tabuarr(r, s) = it + t after the move).
 *   1: the units, in the manner of Zhu et al.'s unit marking (cited in Sec. 3): after the
 *      move of iteration it the two units it moved are marked until it + t, and a move
 *      is tabu while either of the units it would move is marked (mark > it).
 *   2: unit-location pairs, in the manner of Taillard's robust tabu search (cited in
 *      Sec. 4.3): after the move of iteration it each of the two units may not return
 *      to the location it left until it + t, and a move is tabu when both units it
 *      would move would return to such a location.
 * Everything else (tenure, aspiration, best update, early stop, results, trace) is as in
 * orc_tabu, mode 1.  freq (int32[n(n-1)/2]) receives the counts.  Returns 0, or -1 if
 * memory ran out.
 */
ORC_EXPORT int orc_tabu_freq(int n, const int32_t *F, const int32_t *D, const int32_t *p0,
                             int32_t iters, int32_t lo, int32_t hi, uint64_t seed, uint64_t start,
                             int32_t div, int32_t attr, int32_t *best_perm, int64_t *best_cost,
                             int32_t *iters_done, int32_t *freq, int64_t *trace, int32_t trace_cap) {
    int64_t m = (int64_t)n * (n - 1) / 2;
    int64_t *tab = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    int64_t *until = calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int64_t *mark = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));   /* per unit */
    int64_t *uloc = calloc((size_t)(n > 0 ? n * n : 1), sizeof(int64_t)); /* per unit, location */
    int32_t *p = malloc(sizeof(int32_t) * n);
    if (!tab || !until || !mark || !uloc || !p) {
        free(tab); free(until); free(mark); free(uloc); free(p);
        return -1;
    }
    for (int64_t i = 0; i < m; i++) freq[i] = 0;
    memcpy(p, p0, sizeof(int32_t) * n);
    memcpy(best_perm, p0, sizeof(int32_t) * n);
    int64_t cur = orc_cost(n, F, D, p), best = cur;
    int32_t done = 0, last = 0;
    if (m > 0) orc_delta_table(n, F, D, p, tab);
    for (int32_t it = 1; it <= iters && m > 0; it++) {
        int64_t pick = -1;
        /* the tabu attribute of each move at this iteration */
        if (attr == 1) {
            for (int64_t i = 0; i < m; i++) {
                int a, b;
                pair_of(n, i, &a, &b);
                int64_t ma = mark[p[a]], mb = mark[p[b]];
                until[i] = ma > mb ? ma : mb;
            }
        } else if (attr == 2) {
            for (int64_t i = 0; i < m; i++) {
                int a, b;
                pair_of(n, i, &a, &b);
                /* the unit at a would go to b, the one at b to a */
                int64_t xa = uloc[(int64_t)p[a] * n + b], xb = uloc[(int64_t)p[b] * n + a];
                until[i] = xa < xb ? xa : xb;
            }
        }
        int diversify = div > 0 && it - last > div;
        if (diversify) {
            for (int64_t i = 0; i < m; i++) {
                if (until[i] > it) continue;                   /* tabu */
                if (pick < 0 || freq[i] < freq[pick]) pick = i;
            }
            if (pick < 0) diversify = 0;                       /* all tabu: ordinary rule */
        }
        if (!diversify) {
            for (int64_t i = 0; i < m; i++) {
                if (!(until[i] <= it || cur + tab[i] < best)) continue;
                if (pick < 0 || tab[i] < tab[pick]) pick = i;
            }
        }
        if (pick < 0) break;
        int r, s;
        pair_of(n, pick, &r, &s);
        int64_t dz = tab[pick];
        orc_delta_update(n, F, D, p, r, s, tab);
        int32_t tmp = p[r]; p[r] = p[s]; p[s] = tmp;
        cur += dz;
        if (cur < best) { best = cur; memcpy(best_perm, p, sizeof(int32_t) * n); last = it; }
        if (diversify) last = it;
        int64_t tt = (int64_t)it + orc_tenure(seed, (uint64_t)it, start, lo, hi);
        if (attr == 1) { mark[p[r]] = tt; mark[p[s]] = tt; }   /* the units just moved */
        else if (attr == 2) {                                   /* p[s] left r, p[r] left s */
            uloc[(int64_t)p[s] * n + r] = tt;
            uloc[(int64_t)p[r] * n + s] = tt;
        } else until[pick] = tt;
        freq[pick] += 1;
        if (trace && done < trace_cap) {
            trace[4 * done] = r; trace[4 * done + 1] = s;
            trace[4 * done + 2] = dz; trace[4 * done + 3] = cur;
        }
        done = it;
    }
    *best_cost = best;
    if (iters_done) *iters_done = done;
    free(tab); free(until); free(mark); free(uloc); free(p);
    return 0;
}
