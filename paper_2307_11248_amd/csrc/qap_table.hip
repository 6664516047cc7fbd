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

// out[idx(u,v)] = Eq. (2) with the diagonal term for one start, one entry per lane at a
// time (F, D and the permutation already staged).
__device__ void table_body(int n, const uint8_t *Fm, const uint8_t *Dm, const int *perm, int32_t *out);

// table[j][idx(u,v)] for every start j of the launch.
__global__ void __launch_bounds__(256) table_kernel(TableArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const int n = a.n, rs = row_stride(n), job = blockIdx.x, t = threadIdx.x;
    uint8_t *Fm = sm, *Dm = sm + n * rs;
    int *perm = reinterpret_cast<int *>(sm + 2 * n * rs);
    int *pinv = perm + n;
    const bool ok = stage_f_d_perm(a, job, Fm, Dm, perm, pinv, &bad);
    int32_t *out = a.table + (size_t)job * a.m;
    if (!ok) {
        for (int i = t; i < a.m; i += blockDim.x) out[i] = 0;
        return;
    }
    table_body(n, Fm, Dm, perm, out);
}

// The neighbourhood of every item of a batch: block i stages item i's F, D and start.
__global__ void __launch_bounds__(256) table_batch_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const Item &it = b.items[blockIdx.x];
    TableArgs a{it.mats, b.perms + it.perm_off, nullptr, b.table + it.table_off, it.n, it.m, 1};
    const int n = it.n, rs = row_stride(n), t = threadIdx.x;
    uint8_t *Fm = sm, *Dm = sm + n * rs;
    int *perm = reinterpret_cast<int *>(sm + 2 * n * rs);
    int *pinv = perm + n;
    const bool ok = stage_f_d_perm(a, 0, Fm, Dm, perm, pinv, &bad);
    if (!ok) {
        for (int i = t; i < it.m; i += blockDim.x) a.table[i] = 0;
        return;
    }
    table_body(n, Fm, Dm, perm, a.table);
}

// Tables of starting items of a chunked run: block i writes items[i]'s neighbourhood
// into its `table`.
__global__ void __launch_bounds__(256) table_items_kernel(const Item *items) {
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int bad;
    const Item &it = items[blockIdx.x];
    TableArgs a{it.mats, it.perm_in, nullptr, const_cast<int32_t *>(it.table), it.n, it.m, 1};
    const int n = it.n, rs = row_stride(n), t = threadIdx.x;
    uint8_t *Fm = sm, *Dm = sm + n * rs;
    int *perm = reinterpret_cast<int *>(sm + 2 * n * rs);
    int *pinv = perm + n;
    if (!stage_f_d_perm(a, 0, Fm, Dm, perm, pinv, &bad)) {
        for (int i = t; i < it.m; i += blockDim.x) a.table[i] = 0;
        return;
    }
    table_body(n, Fm, Dm, perm, a.table);
}

__device__ void table_body(int n, const uint8_t *Fm, const uint8_t *Dm, const int *perm, int32_t *out) {
    const int rs = row_stride(n), t = threadIdx.x;
    for (int u = 0; u < n - 1; ++u) {
        const int pu = perm[u];
        const long long base = pidx(n, u, u + 1);
        for (int v = u + 1 + t; v < n; v += blockDim.x) {
            const int pv = perm[v];
            const uint8_t *du = Dm + u * rs, *dv = Dm + v * rs;
            const uint8_t *fu = Fm + pu * rs, *fv = Fm + pv * rs;
            int acc = ((int)dv[v] - (int)du[u]) * ((int)fu[pu] - (int)fv[pv])
                    + ((int)dv[u] - (int)du[v]) * ((int)fu[pv] - (int)fv[pu]);
            for (int k = 0; k < n; ++k) {
                if (k == u || k == v) continue;
                const int pk = perm[k];
                const uint8_t *dk = Dm + k * rs, *fk = Fm + pk * rs;
                acc += ((int)dv[k] - (int)du[k]) * ((int)fu[pk] - (int)fv[pk])
                     + ((int)dk[v] - (int)dk[u]) * ((int)fk[pu] - (int)fk[pv]);
            }
            out[base + (v - u - 1)] = acc;
        }
    }
}

size_t table_smem(int n) { return (size_t)2 * n * row_stride(n) + (size_t)2 * n * 4; }

}  // namespace

size_t table_smem_bytes(int n) { return table_smem(n); }

hipError_t launch_table_batch(const BatchArgs &b, size_t smem, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(table_batch_kernel, dim3(b.count), dim3(256), smem, st, b);
    return report(hipGetLastError(), "batch table kernel launch");
}

hipError_t launch_table_items(const Item *d_items, int count, size_t smem, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(table_items_kernel, dim3(count), dim3(256), smem, st, d_items);
    return report(hipGetLastError(), "item table kernel launch");
}

hipError_t launch_cost(const TableArgs &a, hipStream_t st) {
    if (a.k == 0) return hipSuccess;
    const size_t sm = table_smem(a.n);
    hipLaunchKernelGGL(cost_kernel, dim3(a.k), dim3(256), sm, st, a);
    return report(hipGetLastError(), "kernel launch");
}

hipError_t launch_table(const TableArgs &a, hipStream_t st) {
    if (a.k == 0) return hipSuccess;
    const size_t sm = table_smem(a.n);
    hipLaunchKernelGGL(table_kernel, dim3(a.k), dim3(256), sm, st, a);
    return report(hipGetLastError(), "kernel launch");
}

}  // namespace qapk
