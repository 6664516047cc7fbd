// qap_search.hip -- persistent 2opt and tabu search kernels (Secs. 4.1-4.4), one
// workgroup per search, the whole search in one launch.
//
// Data layout
//   * The neighbourhood (one delta per move) lives in registers for the whole search.
//     Lane l of the workgroup owns one tile of the n x n move grid: rows
//     u = ROWS*g .. ROWS*g+ROWS-1 and columns v = 4b .. 4b+3.  Only tiles that hold
//     some u < v are kept.  A tile that straddles the diagonal also holds mirror slots
//     (u > v), which carry the same delta and the same tabu state as (v, u), and
//     diagonal slots (u == v), which hold BIG and are never chosen; slots with u or v
//     beyond n (padding) are reset to BIG after every update.
//   * F, F^T, D, D^T are staged in LDS as u8 rows padded to RS = roundup(n, 16) bytes
//     (F and D only when both are symmetric).
//   * The tabu state of a move is the iteration at which it becomes free again
//     (Tabuarr of Sec. 4.3), one int32 register beside each delta.
//
// One iteration (the move of iteration `it` is chosen from the deltas of the current
// permutation pi; p' = pi with r and s exchanged):
//   select  each lane folds admissibility and a (delta, key) minimum over its slots;
//           wave minimum by shuffles, workgroup minimum through LDS      [barrier B1]
//   A       apply: cost, best-so-far; the four per-index vectors of the incremental
//           update (A, C | B, E packed as int16 pairs); the eight gathered vectors the
//           row recomputation contracts against                          [barrier B2]
//   P       the n-long dot products (u8 x u8, v_dot4) that give, for every u, the
//           deltas of (u, r) and (u, s) under p'                         [barrier B3]
//   R       combine them into Rr[u] = delta'(u, r), Rs[u] = delta'(u, s)   [barrier B4]
//   C       every lane updates its tile: delta += (A_u - A_v)(B_u - B_v)
//           + (C_u - C_v)(E_u - E_v) as one v_pk_sub_i16 pair and one v_dot2; the rows
//           and columns of r and s are overwritten from Rr / Rs; the move gets its tabu
//           tenure.
// The deltas of moves disjoint from {r, s} follow from the k = r, s terms of Eq. (2)
// (Taillard 1991, the elementary tabu search the paper follows); the others are
// recomputed exactly, so every delta stays equal to Eq. (2) of the current permutation.
#include "qap_internal.h"

namespace qapk {

namespace {

typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ inline long long wave_min64(long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline long long wave_sum64(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int pack16(int lo, int hi) {
    return (int)(((unsigned)hi << 16) | ((unsigned)lo & 0xffffu));
}

// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128 multiplications,
// Weyl key schedule.  Returns the first output word.
__device__ inline unsigned long long philox4x64_10_w0(unsigned long long c0, unsigned long long c1,
                                                      unsigned long long c2, unsigned long long c3,
                                                      unsigned long long k0, unsigned long long k1) {
    const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        const unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return c0;
}

// Tenure of the move made at iteration `it` (Sec. 4.3): uniform in [lo, hi].
__device__ inline int draw_tenure(unsigned long long seed, long long it, long long start, int lo, int hi) {
    const unsigned long long x = philox4x64_10_w0((unsigned long long)it, (unsigned long long)start, 0, 0,
                                                  seed, 0);
    const unsigned long long span = (unsigned long long)(long long)(hi - lo + 1);
    return lo + (int)(((x >> 32) * span) >> 32);
}

template <int ROWS>
constexpr int max_lanes() { return ROWS <= 4 ? 1024 : 512; }

template <int ROWS, bool TABU>
__global__ void __launch_bounds__(max_lanes<ROWS>()) search_kernel(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int s_bad;
    const int n = a.n, rs = row_stride(n), L = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wid = t >> 6, W = L >> 6;
    const int job = a.job0 + blockIdx.x;
    const int sym = a.sym;
    const int np = padded_n(n, ROWS);
    const Smem S = smem_plan(n, np, L, sym);

    uint8_t *Fm = sm + S.mats;
    uint8_t *FmT = sym ? Fm : Fm + n * rs;
    uint8_t *Dm = sym ? Fm + n * rs : Fm + 2 * n * rs;
    uint8_t *DmT = sym ? Dm : Fm + 3 * n * rs;
    uint8_t *X = sm + S.x;
    int2 *acbe = reinterpret_cast<int2 *>(sm + S.acbe);
    int2 *R = reinterpret_cast<int2 *>(sm + S.rr);
    int2 *P = reinterpret_cast<int2 *>(sm + S.p);
    int *RD = reinterpret_cast<int *>(sm + S.rd);
    int *CD = reinterpret_cast<int *>(sm + S.cd);
    int *perm = reinterpret_cast<int *>(sm + S.perm);
    int *pinv = reinterpret_cast<int *>(sm + S.pinv);
    int *bestp = reinterpret_cast<int *>(sm + S.bestp);
    int *ten = reinterpret_cast<int *>(sm + S.ten);
    long long *red = reinterpret_cast<long long *>(sm + S.red);

    // ---- stage matrices, clear the gathered vectors, read and check the start
    {
        const int per = n * rs / 16;
        const uint4 *src = reinterpret_cast<const uint4 *>(a.mats);
        uint4 *dst = reinterpret_cast<uint4 *>(Fm);
        const int nm = sym ? 2 : 4;
        for (int mi = 0; mi < nm; ++mi) {
            const int from = sym ? 2 * mi : mi;
            for (int i = t; i < per; i += L) dst[mi * per + i] = src[from * per + i];
        }
        for (int i = t; i < 2 * rs; i += L) reinterpret_cast<int *>(X)[i] = 0;
    }
    if (t == 0) s_bad = 0;
    for (int u = t; u < np; u += L) pinv[u] = -1;
    __syncthreads();
    const int32_t *pin = a.perms_in + (size_t)job * n;
    for (int u = t; u < n; u += L) {
        const int v = pin[u];
        perm[u] = v;
        if (v < 0 || v >= n || atomicExch(&pinv[v], u) != -1) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (a.perm_out != a.perms_in)
            for (int u = t; u < n; u += L) a.perm_out[(size_t)job * n + u] = pin[u];
        if (t == 0) {
            a.cost_out[job] = INT64_MIN;
            if (a.steps_out) a.steps_out[job] = -2;  // QAP_E_NOT_PERM
        }
        return;
    }

    // ---- cost (Eq. 1) and the row/column sums RD_u = sum_k D[u][k] F[p_u][p_k],
    //      CD_u = sum_k D[k][u] F[p_k][p_u] that the row recomputation needs
    long long part = 0;
    for (int u = t; u < n; u += L) {
        bestp[u] = perm[u];
        const uint8_t *fr = Fm + perm[u] * rs, *dr = Dm + u * rs;
        const uint8_t *ftr = FmT + perm[u] * rs, *dtr = DmT + u * rs;
        int acc = 0, acc2 = 0;
        for (int k = 0; k < n; ++k) {
            const int pk = perm[k];
            acc += (int)fr[pk] * (int)dr[k];
            acc2 += (int)ftr[pk] * (int)dtr[k];
        }
        RD[u] = acc;
        CD[u] = acc2;
        part += acc;
    }
    part = wave_sum64(part);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    long long cur = 0;
    for (int w = 0; w < W; ++w) cur += red[w];
    long long best = cur;

    // ---- this lane's tile, its deltas and tabu state
    const bool active = t < a.ntiles;
    int g = 0, b = 0;
    if (active) {
        const int tv = a.tiles[t];
        g = tv & 0xffff;
        b = tv >> 16;
    }
    const int u0 = g * ROWS, v0 = b * TILE_COLS;
    const bool boundary = active && t >= a.ninterior;
    int dl[ROWS][4];
    int ut[TABU ? ROWS : 1][4];
    {
        const int32_t *tab = a.table + (size_t)job * a.m;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = u0 + j, v = v0 + e;
                const bool real = active && u < n && v < n && u != v;
                dl[j][e] = real ? tab[pidx(n, u < v ? u : v, u < v ? v : u)] : BIG;
                if (TABU) ut[j][e] = real ? 0 : INT32_MAX;
            }
        }
    }
    const long long start_id = a.start_base + job;
    int it = 1, steps = 0;
    __syncthreads();

    for (;;) {
        if (TABU) {
            if (it > a.iters) break;
        } else {
            if (steps >= (a.iters > 0 ? a.iters : TWO_OPT_MAX_MOVES)) break;
        }
        // ---- select: lowest (delta, key) over the admissible slots
        int thr = 0;
        if (TABU) {
            const long long d = best - cur;  // aspiration: cur + delta < best
            thr = d < (long long)INT32_MIN ? INT32_MIN : (int)d;
        }
        int bd = INT32_MAX, bs = -1;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = dl[j][e];
                const bool adm = TABU ? (ut[j][e] <= it || x < thr) : true;
                if (adm && x < bd) { bd = x; bs = j * 4 + e; }
            }
        }
        if (!active) bd = INT32_MAX;
        const int key = (bs < 0 || !active) ? KEY_NONE : (((u0 + (bs >> 2)) << 9) | (v0 + (bs & 3)));
        long long kv = ((long long)bd << 32) | (unsigned)key;
        kv = wave_min64(kv);
        if (lane == 0) red[wid] = kv;
        __syncthreads();  // B1
        long long mk = red[0];
        for (int w = 1; w < W; ++w) mk = red[w] < mk ? red[w] : mk;
        const int dstar = (int)(mk >> 32);
        if (TABU ? (dstar == INT32_MAX) : (dstar >= 0)) break;
        const int kstar = (int)(mk & 0xffffffffLL);
        int r = kstar >> 9, s = kstar & 511;
        if (r > s) { const int tmp = r; r = s; s = tmp; }

        // ---- A: apply the move to the cost, build the update vectors
        const int pr = perm[r], ps = perm[s];
        const bool improved = TABU && (cur + dstar < best);
        cur += dstar;
        if (improved) best = cur;
        if (TABU && ((it - 1) % L) == 0) ten[t] = draw_tenure(a.seed, (long long)it + t, start_id, a.lo, a.hi);
        for (int u = t; u < n; u += L) {
            const int pu = perm[u];
            const int A = (int)DmT[r * rs + u] - (int)DmT[s * rs + u];   // d_ur - d_us
            const int Cv = (int)Dm[r * rs + u] - (int)Dm[s * rs + u];    // d_ru - d_su
            const int B = (int)FmT[pr * rs + pu] - (int)FmT[ps * rs + pu];  // f[pu][pr] - f[pu][ps]
            const int E = (int)Fm[pr * rs + pu] - (int)Fm[ps * rs + pu];    // f[pr][pu] - f[ps][pu]
            acbe[u] = make_int2(pack16(A, Cv), pack16(B, E));
            if (u != r && u != s) {
                RD[u] -= A * B;
                CD[u] -= Cv * E;
            }
            const int pu2 = (u == r) ? ps : ((u == s) ? pr : pu);   // p'_u
            // gathered vectors over locations k = u, contracted with rows of D and D^T
            X[4 * rs + u] = Fm[ps * rs + pu2];    // f[p'_r][p'_k]
            X[5 * rs + u] = Fm[pr * rs + pu2];    // f[p'_s][p'_k]
            if (!sym) {
                X[6 * rs + u] = FmT[ps * rs + pu2];  // f[p'_k][p'_r]
                X[7 * rs + u] = FmT[pr * rs + pu2];  // f[p'_k][p'_s]
            }
            // gathered vectors over units m = u, contracted with rows of F and F^T
            const int inv = pinv[u];
            const int inv2 = (u == pr) ? s : ((u == ps) ? r : inv);   // p'^-1(m)
            X[0 * rs + u] = Dm[r * rs + inv2];     // d[r][p'^-1 m]
            X[1 * rs + u] = Dm[s * rs + inv2];     // d[s][p'^-1 m]
            if (!sym) {
                X[2 * rs + u] = DmT[r * rs + inv2];  // d[p'^-1 m][r]
                X[3 * rs + u] = DmT[s * rs + inv2];  // d[p'^-1 m][s]
            }
            if (improved) bestp[u] = pu2;
        }
        __syncthreads();  // B2

        // ---- P: dot products of n-long u8 rows for every u (q: F, F^T, D, D^T rows)
        if (t == 0) {
            perm[r] = ps;
            perm[s] = pr;
            pinv[pr] = s;
            pinv[ps] = r;
        }
        {
            const int nq = sym ? 2 : 4;
            for (int task = t; task < nq * n; task += L) {
                const int qi = task / n, u = task - qi * n;
                const int q = sym ? 2 * qi : qi;
                const int pu2 = (u == r) ? ps : ((u == s) ? pr : perm[u]);
                const uint8_t *row = q == 0 ? Fm + pu2 * rs
                                   : q == 1 ? FmT + pu2 * rs
                                   : q == 2 ? Dm + u * rs : DmT + u * rs;
                const uint8_t *xr = X + (2 * q) * rs, *xs = xr + rs;
                unsigned ar = 0, as = 0;
                for (int w = 0; w < rs; w += 16) {
                    const uint4 rv = *reinterpret_cast<const uint4 *>(row + w);
                    const uint4 x1 = *reinterpret_cast<const uint4 *>(xr + w);
                    const uint4 x2 = *reinterpret_cast<const uint4 *>(xs + w);
                    ar = __builtin_amdgcn_udot4(rv.x, x1.x, ar, false);
                    ar = __builtin_amdgcn_udot4(rv.y, x1.y, ar, false);
                    ar = __builtin_amdgcn_udot4(rv.z, x1.z, ar, false);
                    ar = __builtin_amdgcn_udot4(rv.w, x1.w, ar, false);
                    as = __builtin_amdgcn_udot4(rv.x, x2.x, as, false);
                    as = __builtin_amdgcn_udot4(rv.y, x2.y, as, false);
                    as = __builtin_amdgcn_udot4(rv.z, x2.z, as, false);
                    as = __builtin_amdgcn_udot4(rv.w, x2.w, as, false);
                }
                P[q * np + u] = make_int2((int)ar, (int)as);
            }
        }
        __syncthreads();  // B3

        // ---- R: delta'(u, r) and delta'(u, s) under p' for every u
        {
            const int qF = 0, qFT = sym ? 0 : 1, qD = 2, qDT = sym ? 2 : 3;
            for (int u = t; u < n; u += L) {
                int rr, rsv;
                if (u == r) {
                    rr = BIG;
                    rsv = -dstar;
                } else if (u == s) {
                    rr = -dstar;
                    rsv = BIG;
                } else {
                    const int pa = perm[u];
                    const int daa = Dm[u * rs + u];
                    const int gaa = Fm[pa * rs + pa];
                    const int rdu = RD[u], cdu = CD[u];
                    const int2 p1 = P[qF * np + u], p3 = P[qFT * np + u];
                    const int2 p2 = P[qD * np + u], p4 = P[qDT * np + u];
                    int res[2];
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        const int bb = side ? s : r;
                        const int pb = perm[bb];
                        const int P1 = side ? p1.y : p1.x, P3 = side ? p3.y : p3.x;
                        const int P2 = side ? p2.y : p2.x, P4 = side ? p4.y : p4.x;
                        const int2 rdb2 = P[qD * np + bb], cdb2 = P[qDT * np + bb];
                        const int rdb = side ? rdb2.y : rdb2.x, cdb = side ? cdb2.y : cdb2.x;
                        const int dbb = Dm[bb * rs + bb], dab = Dm[u * rs + bb], dba = Dm[bb * rs + u];
                        const int gbb = Fm[pb * rs + pb], gab = Fm[pa * rs + pb], gba = Fm[pb * rs + pa];
                        const int srow = P1 - rdb - rdu + P2;
                        const int scol = P3 - cdb - cdu + P4;
                        const int rowex = (dba - daa) * (gaa - gba) + (dbb - dab) * (gab - gbb);
                        const int colex = (dab - daa) * (gaa - gab) + (dbb - dba) * (gba - gbb);
                        res[side] = srow + scol - rowex - colex + (dbb - daa) * (gaa - gbb)
                                  + (dba - dab) * (gab - gba);
                    }
                    rr = res[0];
                    rsv = res[1];
                }
                R[u] = make_int2(rr, rsv);
            }
            if (t == 0) {
                RD[r] = P[qD * np + r].x;
                RD[s] = P[qD * np + s].y;
                CD[r] = P[qDT * np + r].x;
                CD[s] = P[qDT * np + s].y;
            }
        }
        __syncthreads();  // B4

        // ---- C: update this lane's tile
        if (active) {
            int acu[ROWS], beu[ROWS], acv[4], bev[4];
#pragma unroll
            for (int j = 0; j < ROWS; ++j) {
                const int2 w = acbe[u0 + j];
                acu[j] = w.x;
                beu[j] = w.y;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int2 w = acbe[v0 + e];
                acv[e] = w.x;
                bev[e] = w.y;
            }
#pragma unroll
            for (int j = 0; j < ROWS; ++j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const short2_t da = __builtin_bit_cast(short2_t, acu[j]) - __builtin_bit_cast(short2_t, acv[e]);
                    const short2_t db = __builtin_bit_cast(short2_t, beu[j]) - __builtin_bit_cast(short2_t, bev[e]);
                    dl[j][e] = __builtin_amdgcn_sdot2(da, db, dl[j][e], false);
                }
            }
            const int rg = r / ROWS, sg = s / ROWS;
            if (g == rg) {
                const int jr = r - u0;
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
                    if (j == jr) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = R[v0 + e].x;
                    }
            }
            if (g == sg) {
                const int js = s - u0;
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
                    if (j == js) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = R[v0 + e].y;
                    }
            }
            if (b == (r >> 2)) {
                const int er = r & 3;
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    const int x = R[u0 + j].x;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e == er) dl[j][e] = x;
                }
            }
            if (b == (s >> 2)) {
                const int es = s & 3;
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    const int x = R[u0 + j].y;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e == es) dl[j][e] = x;
                }
            }
            if (TABU) {
                const int until = it + ten[(it - 1) % L];
                if (g == rg && b == (s >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (j == r - u0 && e == (s & 3)) ut[j][e] = until;
                }
                if (g == sg && b == (r >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (j == s - u0 && e == (r & 3)) ut[j][e] = until;
                }
            }
            if (boundary) {
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (u0 + j >= n || v0 + e >= n) dl[j][e] = BIG;
            }
        }
        if (TABU) ++it; else ++steps;
    }

    // ---- results
    __syncthreads();
    const int *res = TABU ? bestp : perm;
    for (int u = t; u < n; u += L) a.perm_out[(size_t)job * n + u] = res[u];
    if (t == 0) {
        a.cost_out[job] = TABU ? best : cur;
        if (a.steps_out) a.steps_out[job] = TABU ? it - 1 : steps;
    }
}

template <int ROWS, bool TABU>
hipError_t launch_one(const SearchArgs &a, int grid, int lanes, size_t smem, hipStream_t st) {
    hipLaunchKernelGGL((search_kernel<ROWS, TABU>), dim3(grid), dim3(lanes), smem, st, a);
    return report(hipGetLastError(), "kernel launch");
}

}  // namespace

int search_max_lanes(int rows) { return rows <= 4 ? max_lanes<2>() : max_lanes<8>(); }

size_t search_smem_bytes(int n, int rows, int lanes, int sym) {
    return (size_t)smem_plan(n, padded_n(n, rows), lanes, sym).total;
}

hipError_t launch_search(int rows, bool tabu, const SearchArgs &a, int grid, int lanes, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    const size_t smem = search_smem_bytes(a.n, rows, lanes, a.sym);
    switch (rows * 2 + (tabu ? 1 : 0)) {
        case 4: return launch_one<2, false>(a, grid, lanes, smem, st);
        case 5: return launch_one<2, true>(a, grid, lanes, smem, st);
        case 8: return launch_one<4, false>(a, grid, lanes, smem, st);
        case 9: return launch_one<4, true>(a, grid, lanes, smem, st);
        case 16: return launch_one<8, false>(a, grid, lanes, smem, st);
        case 17: return launch_one<8, true>(a, grid, lanes, smem, st);
        case 32: return launch_one<16, false>(a, grid, lanes, smem, st);
        case 33: return launch_one<16, true>(a, grid, lanes, smem, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qapk
