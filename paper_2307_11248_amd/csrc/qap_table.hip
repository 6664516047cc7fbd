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

// Neighbourhood row r of start `job` (block (r, job)): wave w evaluates the exchanges of
// locations r and s = r + 1 + w, r + 1 + w + W, ... by Eq. (2), with G = F[p][p]:
//   delta(r, s) = sum_{k != r, s} (G_sk - G_rk)(D_rk - D_sk) + (G_ks - G_kr)(D_kr - D_ks)
//               + (G_ss - G_rr)(D_rr - D_ss) + (G_sr - G_rs)(D_rs - D_sr),
// its 64 lanes splitting k (so each row of F, F^T, D, D^T at s is read by one wave, in
// one contiguous stretch) and summing their parts at the end.  Row r's bytes (G_rk, G_kr,
// D_rk, D_kr) are staged in LDS.
__global__ void __launch_bounds__(TB_LANES) table_wide_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const int n = a.n, rs = row_stride(n), r = blockIdx.x, job = blockIdx.y, t = threadIdx.x;
    int32_t *out = a.table + (size_t)job * a.m;
    int *perm = reinterpret_cast<int *>(sm), *pinv = perm + n;
    uint8_t *gr = reinterpret_cast<uint8_t *>(pinv + n), *gtr = gr + n, *dr = gtr + n, *dtr = dr + n;
    const int s = r + 1 + t;
    if (!tb_stage_perm(a.perms + (size_t)job * n, n, perm, pinv, &bad)) {
        if (s < n) out[pidx(n, r, s)] = 0;
        return;
    }
    const uint8_t *F = a.mats, *FT = F + (size_t)n * rs, *D = F + (size_t)2 * n * rs, *DT = F + (size_t)3 * n * rs;
    const int pr = perm[r];
    for (int k = t; k < n; k += blockDim.x) {
        const int pk = perm[k];
        gr[k] = F[(size_t)pr * rs + pk];
        gtr[k] = FT[(size_t)pr * rs + pk];
        dr[k] = D[(size_t)r * rs + k];
        dtr[k] = DT[(size_t)r * rs + k];
    }
    __syncthreads();
    const int lane = t & 63, W = blockDim.x >> 6;
    for (int sw = r + 1 + (t >> 6); sw < n; sw += W) {
        const int ps = perm[sw];
        const uint8_t *Fs = F + (size_t)ps * rs, *FTs = FT + (size_t)ps * rs, *Ds = D + (size_t)sw * rs,
                      *DTs = DT + (size_t)sw * rs;
        int acc = 0;
        for (int k = lane; k < n; k += 64) {
            const int pk = perm[k];
            const int term = ((int)Fs[pk] - (int)gr[k]) * ((int)dr[k] - (int)Ds[k]) +
                             ((int)FTs[pk] - (int)gtr[k]) * ((int)dtr[k] - (int)DTs[k]);
            acc += (k == r || k == sw) ? 0 : term;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0)
            out[pidx(n, r, sw)] = acc + ((int)Fs[ps] - (int)gr[r]) * ((int)dr[r] - (int)Ds[sw]) +
                                  ((int)Fs[pr] - (int)gr[sw]) * ((int)dr[sw] - (int)Ds[r]);
    }
}

// (I, J), I <= J, of tile pair q in row-major order over nt x nt tiles
__device__ inline void tb_pair(int q, int nt, int &I, int &J) {
    I = 0;
    while (q >= nt - I) {
        q -= nt - I;
        ++I;
    }
    J = I + q;
}

__device__ inline long long tb_load8(const uint8_t *p) { return *reinterpret_cast<const long long *>(p); }

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
        for (int j0 = 0; j0 < a.k; j0 += 65535) {
            TableArgs b = a;
            b.perms += (size_t)j0 * a.n;
            b.table += (size_t)j0 * a.m;
            b.k = a.k - j0 < 65535 ? a.k - j0 : 65535;
            hipLaunchKernelGGL(table_wide_kernel, dim3(a.n - 1, b.k), dim3(TB_LANES), (size_t)2 * a.n * 4 + 4 * a.n,
                               st, b);
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
