// qap_table.hip -- cost (Eq. 1) and whole-neighbourhood (Eq. 2) kernels.
//
// One workgroup per start.  F and D are staged in LDS as u8 (every entry lies in
// [0, 255]); the start's permutation and its inverse are staged beside them.
#include "qap_internal.h"

namespace qapk {

namespace {

__device__ inline long long wave_sum64(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Stage F and D (global matrices 0 and 2) and one permutation; returns false if the row
// is not a permutation of 0..n-1.  Ends with a barrier.
__device__ bool stage_f_d_perm(const TableArgs &a, int job, uint8_t *Fm, uint8_t *Dm, int *perm,
                               int *pinv, int *bad) {
    const int n = a.n, rs = row_stride(n), L = blockDim.x, t = threadIdx.x;
    const int per = n * rs / 16;
    const uint4 *src = reinterpret_cast<const uint4 *>(a.mats);
    for (int i = t; i < per; i += L) {
        reinterpret_cast<uint4 *>(Fm)[i] = src[i];
        reinterpret_cast<uint4 *>(Dm)[i] = src[2 * per + i];
    }
    if (t == 0) *bad = 0;
    for (int u = t; u < n; u += L) pinv[u] = -1;
    __syncthreads();
    const int32_t *p = a.perms + (size_t)job * n;
    for (int u = t; u < n; u += L) {
        const int v = p[u];
        perm[u] = v;
        if (v < 0 || v >= n || atomicExch(&pinv[v], u) != -1) *bad = 1;
    }
    __syncthreads();
    return *bad == 0;
}

// costs[j] = sum_i sum_k F[p_i][p_k] D[i][k]   (Eq. 1)
__global__ void __launch_bounds__(256) cost_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    __shared__ long long red[4];
    const int n = a.n, rs = row_stride(n), job = blockIdx.x, t = threadIdx.x;
    uint8_t *Fm = sm, *Dm = sm + n * rs;
    int *perm = reinterpret_cast<int *>(sm + 2 * n * rs);
    int *pinv = perm + n;
    const bool ok = stage_f_d_perm(a, job, Fm, Dm, perm, pinv, &bad);
    if (!ok) {
        if (t == 0) a.costs[job] = INT64_MIN;
        return;
    }
    long long part = 0;
    for (int i = t; i < n; i += blockDim.x) {
        const uint8_t *frow = Fm + perm[i] * rs, *drow = Dm + i * rs;
        int acc = 0;
        for (int k = 0; k < n; ++k) acc += (int)frow[perm[k]] * (int)drow[k];
        part += acc;
    }
    part = wave_sum64(part);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    if (t == 0) {
        long long z = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) z += red[w];
        a.costs[job] = z;
    }
}

// ---- whole neighbourhood (a3) as integer contractions on the matrix cores
//
// With G = F[p][p] (G[a][b] = F[p_a][p_b]) and T = G.D^T + G^T.D, every delta of Eq. (2)
// (with its diagonal term) is
//   delta(i, j) = T_ij + T_ji - T_ii - T_jj + c_ij,
// c_ij a sum of six products of the entries of D and G at (i, j), (j, i), (i, i), (j, j)
// (expanding Eq. (2) and collecting the k = i, j terms).  The two n x n x n products
// run as v_mfma_i32_32x32x16_i8 on entries shifted to int8 (x - 128), with the shift
// undone exactly from row sums:
//   sum_k x_k y_k = sum_k x'_k y'_k + 128 (sum_k x'_k + sum_k y'_k) + 128^2 n.
// A workgroup takes one start.  Phase 0 stages X = G', Y = D' (int8, rows padded to a
// multiple of 32 with zeros) in LDS, phase 1 X = (G^T)', Y = (D^T)' (skipped when F and
// D are both symmetric: then the phases are equal).  Each wave owns pairs of 32 x 32
// output tiles (I <= J) and accumulates S_ij = T_ij + T_ji in place as
// X_I.Y_J^T + Y_I.X_J^T over both phases, so the transpose costs nothing.

typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int TB_LANES = 512, TB_W = TB_LANES / 64;
constexpr int TB_MAXP = 5;   // tile pairs per wave: 36 pairs at n = 256 over 8 waves

__host__ __device__ inline int tb_rows(int n) { return (n + 31) & ~31; }

struct TbPlan {
    int perm, pinv, x, y, u, td, total;
};

__host__ __device__ inline TbPlan tb_plan(int n) {
    const int rs = row_stride(n), np = tb_rows(n);
    TbPlan q;
    int o = 0;
    q.perm = o; o += np * 4;
    q.pinv = o; o += np * 4;
    q.u = o;    o += np * 4;
    q.td = o;   o += np * 4;
    o = (o + 255) & ~255;
    q.x = o;    o += np * rs;
    o = (o + 255) & ~255;
    q.y = o;    o += np * rs;
    q.total = o;
    return q;
}

// Read and check one start into LDS (perm and its inverse); false if it is not a
// permutation of 0..n-1.  Ends with a barrier.
__device__ bool tb_stage_perm(const int32_t *p, int n, int *perm, int *pinv, int *bad) {
    const int L = blockDim.x, t = threadIdx.x;
    if (t == 0) *bad = 0;
    for (int u = t; u < n; u += L) pinv[u] = -1;
    __syncthreads();
    for (int u = t; u < n; u += L) {
        const int v = p[u];
        perm[u] = v;
        if (v < 0 || v >= n || atomicExch(&pinv[v], u) != -1) *bad = 1;
    }
    __syncthreads();
    return *bad == 0;
}

// n above WIDE_N (F and D do not fit in LDS): the matrices are read in place from global
// memory, only the start and its inverse are staged.

// Cost (Eq. 1) of one start per workgroup.
__global__ void __launch_bounds__(256) cost_wide_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    __shared__ long long red[4];
    const int n = a.n, rs = row_stride(n), job = blockIdx.x, t = threadIdx.x;
    int *perm = reinterpret_cast<int *>(sm), *pinv = perm + n;
    if (!tb_stage_perm(a.perms + (size_t)job * n, n, perm, pinv, &bad)) {
        if (t == 0) a.costs[job] = INT64_MIN;
        return;
    }
    const uint8_t *F = a.mats, *D = a.mats + (size_t)2 * n * rs;
    long long part = 0;
    for (int i = t; i < n; i += blockDim.x) {
        const uint8_t *frow = F + (size_t)perm[i] * rs, *drow = D + (size_t)i * rs;
        int acc = 0;   // at most n * 255^2 < 2^31
        for (int k = 0; k < n; ++k) acc += (int)frow[perm[k]] * (int)drow[k];
        part += acc;
    }
    part = wave_sum64(part);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    if (t == 0) {
        long long z = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) z += red[w];
        a.costs[job] = z;
    }
}

// (I, J), I <= J, of pair q in row-major order over nt x nt
__device__ inline void tb_pair(int q, int nt, int &I, int &J) {
    I = 0;
    while (q >= nt - I) {
        q -= nt - I;
        ++I;
    }
    J = I + q;
}

__device__ inline long long tb_load8(const uint8_t *p) { return *reinterpret_cast<const long long *>(p); }

// ---- whole neighbourhood above WIDE_N: the same contraction, blocked
//
// X = G' and Y = D' no longer fit in LDS for a whole start, so a workgroup takes one pair
// (BI <= BJ) of 128-row blocks of one start and streams k through LDS in chunks of
// TW_KC: each chunk stages X and Y of both row blocks (X gathered from global F through
// the permutation, Y read from global D, both shifted to int8), adds its part of the row
// sums and diagonal terms of those rows, and accumulates the 32 x 32 output tiles of the
// pair (two per wave) with v_mfma_i32_32x32x16_i8.  The epilogue is the one of the
// single-block kernel, with the entries of D and G at (i, j), (j, i), (i, i), (j, j)
// read from global memory.

constexpr int TW_ROWS = 128;                 // rows of a block
constexpr int TW_KC = 128;                   // k per chunk
constexpr int TW_RS = TW_KC + 16;            // LDS row stride of a staged chunk
constexpr int TW_TILES = TW_ROWS / 32;       // 32 x 32 tiles per block side

struct TwPlan {
    int perm, xi, yi, xj, yj, ui, uj, ti, tj, total;
};

__host__ __device__ inline TwPlan tw_plan(int n) {
    TwPlan q;
    int o = 0;
    q.perm = o; o += ((n + 3) & ~3) * 4;
    o = (o + 255) & ~255;
    q.xi = o; o += TW_ROWS * TW_RS;
    q.yi = o; o += TW_ROWS * TW_RS;
    q.xj = o; o += TW_ROWS * TW_RS;
    q.yj = o; o += TW_ROWS * TW_RS;
    q.ui = o; o += TW_ROWS * 4;
    q.uj = o; o += TW_ROWS * 4;
    q.ti = o; o += TW_ROWS * 4;
    q.tj = o; o += TW_ROWS * 4;
    q.total = o;
    return q;
}

__global__ void __launch_bounds__(TB_LANES) table_wide_mfma_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const int n = a.n, rs = row_stride(n), job = blockIdx.y, t = threadIdx.x, L = blockDim.x;
    const int lane = t & 63, w = t >> 6;
    const TwPlan P = tw_plan(n);
    int32_t *out = a.table + (size_t)job * a.m;
    int *perm = reinterpret_cast<int *>(sm + P.perm);
    int *U_i = reinterpret_cast<int *>(sm + P.ui), *U_j = reinterpret_cast<int *>(sm + P.uj);
    int *T_i = reinterpret_cast<int *>(sm + P.ti), *T_j = reinterpret_cast<int *>(sm + P.tj);
    uint8_t *Xi = sm + P.xi, *Yi = sm + P.yi, *Xj = sm + P.xj, *Yj = sm + P.yj;
    const int nb = (n + TW_ROWS - 1) / TW_ROWS;
    int BI, BJ;
    tb_pair(blockIdx.x, nb, BI, BJ);
    const bool same = BI == BJ;
    // check the start (its inverse in the X chunk buffer, which is free until staging)
    {
        int *pinv = reinterpret_cast<int *>(Xi);
        if (t == 0) bad = 0;
        for (int u = t; u < n; u += L) pinv[u] = -1;
        __syncthreads();
        const int32_t *p = a.perms + (size_t)job * n;
        for (int u = t; u < n; u += L) {
            const int v = p[u];
            perm[u] = v;
            if (v < 0 || v >= n || atomicExch(&pinv[v], u) != -1) bad = 1;
        }
        __syncthreads();
        if (bad) {
            // every block of the start clears its own entries
            for (int x = t; x < TW_ROWS * TW_ROWS; x += L) {
                const int i = BI * TW_ROWS + x / TW_ROWS, j = BJ * TW_ROWS + x % TW_ROWS;
                if (i < j && j < n) out[pidx(n, i, j)] = 0;
            }
            return;
        }
    }
    for (int x = t; x < TW_ROWS; x += L) U_i[x] = U_j[x] = T_i[x] = T_j[x] = 0;

    // the wave's output tiles: (ti, tj) in the pair, ti <= tj when the blocks are the same
    const int ntiles = same ? TW_TILES * (TW_TILES + 1) / 2 : TW_TILES * TW_TILES;
    int tI[2], tJ[2];
    bool has[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int id = w + 8 * q;
        has[q] = id < ntiles;
        if (same) {
            tb_pair(has[q] ? id : 0, TW_TILES, tI[q], tJ[q]);
        } else {
            tI[q] = id / TW_TILES;
            tJ[q] = id % TW_TILES;
        }
    }
    v16i acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0;

    // per row of the two blocks (threads 0 .. 2 TW_ROWS - 1): sum x', sum y', sum x y
    int sx = 0, sy = 0, dxy = 0, u_acc = 0, t_acc = 0;
    const int phases = a.sym ? 1 : 2;
    const int wpr = TW_KC / 4;   // words per staged row
    for (int ph = 0; ph < phases; ++ph) {
        const uint8_t *Fp = a.mats + (size_t)(ph ? 1 : 0) * n * rs;   // F, then F^T
        const uint8_t *Dp = a.mats + (size_t)(ph ? 3 : 2) * n * rs;   // D, then D^T
        sx = sy = dxy = 0;
        for (int k0 = 0; k0 < n; k0 += TW_KC) {
            __syncthreads();   // the previous chunk is consumed
            const int sides = same ? 1 : 2;
            for (int v = t; v < sides * TW_ROWS * wpr; v += L) {
                const int side = v / (TW_ROWS * wpr), rem = v - side * TW_ROWS * wpr;
                const int ri = rem / wpr, c = (rem - ri * wpr) * 4;
                const int i = (side ? BJ : BI) * TW_ROWS + ri, k = k0 + c;
                unsigned xw = 0, yw = 0;
                if (i < n) {
                    const uint8_t *frow = Fp + (size_t)perm[i] * rs, *drow = Dp + (size_t)i * rs;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (k + e < n) {
                            xw |= (unsigned)(frow[perm[k + e]] ^ 0x80u) << (8 * e);
                            yw |= (unsigned)(drow[k + e] ^ 0x80u) << (8 * e);
                        }
                }
                reinterpret_cast<unsigned *>(side ? Xj : Xi)[(ri * TW_RS + c) / 4] = xw;
                reinterpret_cast<unsigned *>(side ? Yj : Yi)[(ri * TW_RS + c) / 4] = yw;
            }
            __syncthreads();
            // row sums and diagonal terms of this chunk
            if (t < (same ? 1 : 2) * TW_ROWS) {
                const int side = t / TW_ROWS, ri = t - side * TW_ROWS;
                const int *xr = reinterpret_cast<const int *>((side ? Xj : Xi) + ri * TW_RS);
                const int *yr = reinterpret_cast<const int *>((side ? Yj : Yi) + ri * TW_RS);
                for (int c = 0; c < wpr; ++c) {
                    sx = __builtin_amdgcn_sdot4(xr[c], 0x01010101, sx, false);
                    sy = __builtin_amdgcn_sdot4(yr[c], 0x01010101, sy, false);
                    dxy = __builtin_amdgcn_sdot4(xr[c], yr[c], dxy, false);
                }
            }
            // S += X_I . Y_J^T + Y_I . X_J^T over this chunk
            const int row = lane & 31, kh = 8 * (lane >> 5);
            const uint8_t *XJ = same ? Xi : Xj, *YJ = same ? Yi : Yj;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (!has[q]) continue;
                const uint8_t *xi = Xi + (tI[q] * 32 + row) * TW_RS + kh, *yj = YJ + (tJ[q] * 32 + row) * TW_RS + kh;
                const uint8_t *yi = Yi + (tI[q] * 32 + row) * TW_RS + kh, *xj = XJ + (tJ[q] * 32 + row) * TW_RS + kh;
#pragma unroll
                for (int kk = 0; kk < TW_KC; kk += 16) {
                    acc[q] = __builtin_amdgcn_mfma_i32_32x32x16_i8(tb_load8(xi + kk), tb_load8(yj + kk), acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_i32_32x32x16_i8(tb_load8(yi + kk), tb_load8(xj + kk), acc[q], 0, 0, 0);
                }
            }
        }
        // this phase's share of the row sums and diagonal terms
        u_acc += sx + sy;
        t_acc += dxy + 128 * (sx + sy) + 16384 * n;
    }
    if (t < (same ? 1 : 2) * TW_ROWS) {
        const int side = t / TW_ROWS, ri = t - side * TW_ROWS;
        (side ? U_j : U_i)[ri] = u_acc;
        (side ? T_j : T_i)[ri] = t_acc;
    }
    __syncthreads();
    const int *UJ = same ? U_i : U_j, *TJ = same ? T_i : T_j;

    // ---- epilogue: delta(i, j) for i < j of the wave's tiles
    const uint8_t *F = a.mats, *FT = F + (size_t)n * rs, *D = F + (size_t)2 * n * rs, *DT = F + (size_t)3 * n * rs;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (!has[q]) continue;
        const int jl = tJ[q] * 32 + (lane & 31), j = BJ * TW_ROWS + jl;
        if (j >= n) continue;
        const int pj = perm[j];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int il = tI[q] * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), i = BI * TW_ROWS + il;
            if (i < j) {
                const int pi = perm[i];
                const int s_ij = a.sym ? 2 * (acc[q][r] + 128 * (U_i[il] + UJ[jl]) + 32768 * n)
                                       : acc[q][r] + 128 * (U_i[il] + UJ[jl]) + 65536 * n;
                const int t_ii = a.sym ? 2 * T_i[il] : T_i[il], t_jj = a.sym ? 2 * TJ[jl] : TJ[jl];
                const int Dij = D[(size_t)i * rs + j], Dji = DT[(size_t)i * rs + j];
                const int Dii = D[(size_t)i * rs + i], Djj = D[(size_t)j * rs + j];
                const int Gij = F[(size_t)pi * rs + pj], Gji = FT[(size_t)pi * rs + pj];
                const int Gii = F[(size_t)pi * rs + pi], Gjj = F[(size_t)pj * rs + pj];
                const int c = -(Dji - Dii) * (Gii - Gji) - (Djj - Dij) * (Gij - Gjj) - (Dij - Dii) * (Gii - Gij)
                              - (Djj - Dji) * (Gji - Gjj) + (Dji - Dij) * (Gij - Gji) + (Djj - Dii) * (Gii - Gjj);
                out[pidx(n, i, j)] = s_ij - t_ii - t_jj + c;
            }
        }
    }
}


// The whole neighbourhood of one start, perm already in LDS (tb_plan layout at sm).
__device__ __attribute__((always_inline)) void table_mfma_body(const uint8_t *mats, int n, int sym, unsigned char *sm, int32_t *out) {
    const TbPlan P = tb_plan(n);
    const int rs = row_stride(n), np = tb_rows(n), nt = np / 32, L = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int *perm = reinterpret_cast<const int *>(sm + P.perm);
    int *U = reinterpret_cast<int *>(sm + P.u);
    int *TD = reinterpret_cast<int *>(sm + P.td);
    uint8_t *X = sm + P.x, *Y = sm + P.y;
    const int npairs = nt * (nt + 1) / 2;
    for (int i = t; i < np; i += L) U[i] = TD[i] = 0;

    v16i acc[TB_MAXP];
#pragma unroll
    for (int q = 0; q < TB_MAXP; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0;

    const int phases = sym ? 1 : 2;
    for (int ph = 0; ph < phases; ++ph) {
        const uint8_t *Fp = mats + (size_t)(ph ? 1 : 0) * n * rs;   // F, then F^T
        const uint8_t *Dp = mats + (size_t)(ph ? 3 : 2) * n * rs;   // D, then D^T
        // raw rows of F_p into Y, then X[i][k] = F_p[p_i][p_k] - 128 gathered from them
        const int vec = n * rs / 16;
        for (int v = t; v < vec; v += L)
            reinterpret_cast<uint4 *>(Y)[v] = reinterpret_cast<const uint4 *>(Fp)[v];
        __syncthreads();
        const int wpr = rs / 4;
        for (int v = t; v < np * wpr; v += L) {
            const int i = v / wpr, k0 = (v - i * wpr) * 4;
            unsigned word = 0;
            if (i < n) {
                const uint8_t *row = Y + perm[i] * rs;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (k0 + e < n) word |= (unsigned)(row[perm[k0 + e]] ^ 0x80u) << (8 * e);
            }
            reinterpret_cast<unsigned *>(X)[v] = word;
        }
        __syncthreads();
        // Y[i][k] = D_p[i][k] - 128 (the global rows are zero past n: shift real bytes only)
        const int vpr = rs / 16;
        for (int v = t; v < np * vpr; v += L) {
            const int i = v / vpr, c = (v - i * vpr) * 16;
            uint4 x = make_uint4(0, 0, 0, 0);
            if (i < n) {
                x = reinterpret_cast<const uint4 *>(Dp + (size_t)i * rs)[c / 16];
                unsigned m[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = c + 4 * e, real = n - k;   // bytes k .. k+3, real ones first
                    m[e] = real >= 4 ? 0x80808080u : (real <= 0 ? 0u : (0x80808080u >> (8 * (4 - real))));
                }
                x.x ^= m[0]; x.y ^= m[1]; x.z ^= m[2]; x.w ^= m[3];
            }
            reinterpret_cast<uint4 *>(Y)[v] = x;
        }
        __syncthreads();
        // per index: the row sums of X' and Y' and the diagonal term sum_k x_ik y_ik
        for (int i = t; i < n; i += L) {
            const int *xr = reinterpret_cast<const int *>(X + i * rs), *yr = reinterpret_cast<const int *>(Y + i * rs);
            int sx = 0, sy = 0, dxy = 0;
            for (int c = 0; c < rs / 4; ++c) {
                const int a = xr[c], b = yr[c];
                sx = __builtin_amdgcn_sdot4(a, 0x01010101, sx, false);
                sy = __builtin_amdgcn_sdot4(b, 0x01010101, sy, false);
                dxy = __builtin_amdgcn_sdot4(a, b, dxy, false);
            }
            U[i] += sx + sy;
            TD[i] += dxy + 128 * (sx + sy) + 16384 * n;
        }
        // S += X_I . Y_J^T + Y_I . X_J^T over this phase
        const int row = lane & 31, kh = 8 * (lane >> 5);
#pragma unroll
        for (int q = 0; q < TB_MAXP; ++q) {
            const int pq = w + q * TB_W;
            if (pq < npairs) {
                int I, J;
                tb_pair(pq, nt, I, J);
                const uint8_t *xi = X + (I * 32 + row) * rs + kh, *yj = Y + (J * 32 + row) * rs + kh;
                const uint8_t *yi = Y + (I * 32 + row) * rs + kh, *xj = X + (J * 32 + row) * rs + kh;
                for (int k0 = 0; k0 < n; k0 += 16) {
                    acc[q] = __builtin_amdgcn_mfma_i32_32x32x16_i8(tb_load8(xi + k0), tb_load8(yj + k0), acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_i32_32x32x16_i8(tb_load8(yi + k0), tb_load8(xj + k0), acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // sums visible; X, Y free for the next phase
    }

    // ---- epilogue: delta(i, j) for i < j from the accumulators of this wave.  X and Y
    //      hold the last phase: G^T and D^T (or G and D when symmetric, then equal to them
    //      transposed), so G_ab = X[b][a] + 128 and D_ab = Y[b][a] + 128 in both cases.
    auto gv = [&](int a_, int b_) { return (int)(uint8_t)(X[b_ * rs + a_] ^ 0x80); };
    auto dv = [&](int a_, int b_) { return (int)(uint8_t)(Y[b_ * rs + a_] ^ 0x80); };
#pragma unroll
    for (int q = 0; q < TB_MAXP; ++q) {
        const int pq = w + q * TB_W;
        if (pq >= npairs) continue;
        int I, J;
        tb_pair(pq, nt, I, J);
        const int j = J * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = I * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (i < j && j < n) {
                const int s_ij = sym ? 2 * (acc[q][r] + 128 * (U[i] + U[j]) + 32768 * n)
                                     : acc[q][r] + 128 * (U[i] + U[j]) + 65536 * n;
                const int t_ii = sym ? 2 * TD[i] : TD[i], t_jj = sym ? 2 * TD[j] : TD[j];
                const int Dij = dv(i, j), Dji = dv(j, i), Dii = dv(i, i), Djj = dv(j, j);
                const int Gij = gv(i, j), Gji = gv(j, i), Gii = gv(i, i), Gjj = gv(j, j);
                const int c = -(Dji - Dii) * (Gii - Gji) - (Djj - Dij) * (Gij - Gjj) - (Dij - Dii) * (Gii - Gij)
                              - (Djj - Dji) * (Gji - Gjj) + (Dji - Dij) * (Gij - Gji) + (Djj - Dii) * (Gii - Gjj);
                out[pidx(n, i, j)] = s_ij - t_ii - t_jj + c;
            }
        }
    }
}

// table[j][idx(u,v)] for every start j of the launch.
__global__ void __launch_bounds__(TB_LANES) table_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const TbPlan P = tb_plan(a.n);
    const int job = blockIdx.x, t = threadIdx.x;
    int32_t *out = a.table + (size_t)job * a.m;
    if (!tb_stage_perm(a.perms + (size_t)job * a.n, a.n, reinterpret_cast<int *>(sm + P.perm),
                       reinterpret_cast<int *>(sm + P.pinv), &bad)) {
        for (int i = t; i < a.m; i += blockDim.x) out[i] = 0;
        return;
    }
    table_mfma_body(a.mats, a.n, a.sym, sm, out);
}

// The neighbourhood of every item of a batch: block i takes item i's start.
__global__ void __launch_bounds__(TB_LANES) table_batch_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const Item &it = b.items[blockIdx.x];
    const TbPlan P = tb_plan(it.n);
    int32_t *out = b.table + it.table_off;
    if (!tb_stage_perm(b.perms + it.perm_off, it.n, reinterpret_cast<int *>(sm + P.perm),
                       reinterpret_cast<int *>(sm + P.pinv), &bad)) {
        for (int i = threadIdx.x; i < it.m; i += blockDim.x) out[i] = 0;
        return;
    }
    table_mfma_body(it.mats, it.n, it.sym, sm, out);
}

// Tables of starting items of a chunked run: block i writes items[i]'s neighbourhood
// into its `table`.
__global__ void __launch_bounds__(TB_LANES) table_items_kernel(const Item *items) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const Item &it = items[blockIdx.x];
    const TbPlan P = tb_plan(it.n);
    int32_t *out = const_cast<int32_t *>(it.table);
    if (!tb_stage_perm(it.perm_in, it.n, reinterpret_cast<int *>(sm + P.perm), reinterpret_cast<int *>(sm + P.pinv),
                       &bad)) {
        for (int i = threadIdx.x; i < it.m; i += blockDim.x) out[i] = 0;
        return;
    }
    table_mfma_body(it.mats, it.n, it.sym, sm, out);
}

size_t table_smem(int n) { return (size_t)tb_plan(n).total; }

size_t cost_smem(int n) { return (size_t)2 * n * row_stride(n) + (size_t)2 * n * 4; }

}  // namespace

size_t table_smem_bytes(int n) { return table_smem(n); }

hipError_t launch_table_batch(const BatchArgs &b, size_t smem, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(table_batch_kernel, dim3(b.count), dim3(TB_LANES), smem, st, b);
    return report(hipGetLastError(), "batch table kernel launch");
}

hipError_t launch_table_items(const Item *d_items, int count, size_t smem, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(table_items_kernel, dim3(count), dim3(TB_LANES), smem, st, d_items);
    return report(hipGetLastError(), "item table kernel launch");
}

hipError_t launch_cost(const TableArgs &a, hipStream_t st) {
    if (a.k == 0) return hipSuccess;
    if (a.n > WIDE_N) {
        hipLaunchKernelGGL(cost_wide_kernel, dim3(a.k), dim3(256), (size_t)2 * a.n * 4, st, a);
        return report(hipGetLastError(), "kernel launch");
    }
    const size_t sm = cost_smem(a.n);
    hipLaunchKernelGGL(cost_kernel, dim3(a.k), dim3(256), sm, st, a);
    return report(hipGetLastError(), "kernel launch");
}

hipError_t launch_table(const TableArgs &a, hipStream_t st) {
    if (a.k == 0) return hipSuccess;
    if (a.n > WIDE_N) {   // starts in groups of at most 65535 (the grid's y extent)
        const int nb = (a.n + TW_ROWS - 1) / TW_ROWS;
        for (int j0 = 0; j0 < a.k; j0 += 65535) {
            TableArgs b = a;
            b.perms += (size_t)j0 * a.n;
            b.table += (size_t)j0 * a.m;
            b.k = a.k - j0 < 65535 ? a.k - j0 : 65535;
            hipLaunchKernelGGL(table_wide_mfma_kernel, dim3(nb * (nb + 1) / 2, b.k), dim3(TB_LANES),
                               (size_t)tw_plan(a.n).total, st, b);
            const hipError_t e = report(hipGetLastError(), "kernel launch");
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const size_t sm = table_smem(a.n);
    hipLaunchKernelGGL(table_kernel, dim3(a.k), dim3(TB_LANES), sm, st, a);
    return report(hipGetLastError(), "kernel launch");
}

}  // namespace qapk
