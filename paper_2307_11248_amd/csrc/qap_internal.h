// qap_internal.h -- device helpers, shared-memory plan and launch declarations of libqap.
// Internal to the library: the public ABI is include/qap.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstdio>
#include <cstdlib>

namespace qapk {

// Delta held by slots that are not moves (the diagonal u == v of a tile and padding
// beyond n).  Larger than any real delta (|delta| <= (2n - 2) * 255^2 < 2^26 for entries
// in [0, 255] and n <= 512), so such a slot is never the best candidate, and the
// incremental update adds exactly 0 to a diagonal slot.
constexpr int BIG = 0x3FFFFFFF;
constexpr int KEY_NONE = 0x7FFFFFFF;
constexpr int TILE_COLS = 4;   // columns of the register tile held by one lane
// Above this n, G = F[p][p] and G^T no longer fit in LDS beside the search's other
// arrays: the wide streamed kernel keeps them, like D and D^T, in global memory.
constexpr int WIDE_N = 256;
// Moves of one 2opt search run to a local optimum (max_iters <= 0): unbounded in effect.
// The integer cost strictly decreases with every move, so the search always ends at a
// local optimum; the bound only keeps the move counter inside int32.
constexpr int TWO_OPT_MAX_MOVES = INT32_MAX;

// Rows are padded to RS bytes, an odd multiple of 16 (16 more than n rounded up to 32):
// every row starts 16-byte aligned, 16 consecutive rows start in 16 different groups of
// four LDS banks, so the 16-byte row reads of a wave (one row per index) do not
// collide, and the zero padding covers n rounded up to 32, so row dot products may
// step 32 bytes at a time.
__host__ __device__ inline int row_stride(int n) { return ((n + 31) & ~31) + 16; }

// Number of indices (locations or units) addressable by a tile of `rows` x 4.
__host__ __device__ inline int padded_n(int n, int rows) {
    int a = ((n + rows - 1) / rows) * rows;
    int b = ((n + TILE_COLS - 1) / TILE_COLS) * TILE_COLS;
    int m = a > b ? a : b;
    return (m + 3) & ~3;
}

__host__ __device__ inline long long pidx(int n, int r, int s) {
    return (long long)r * n - (long long)r * (r + 1) / 2 + (s - r - 1);
}

// Lanes a search workgroup needs: one per register tile, and at least one per (index,
// dot family) task when that fits, so the row recomputation runs in one pass.
__host__ __device__ inline int families(int sym) { return sym ? 2 : 4; }

// Byte offsets of the per-search shared-memory arrays of the search kernels.  The
// matrices are u8 rows of RS bytes: D, D^T, and G = F[p][p] (the flows seen from the
// locations under the current permutation p), G^T; only D and G when F and D are
// both symmetric.
struct Smem {
    int d, dt, g, gt, acbe, rpr, rps, kc, perm, bestp, pinv, ten, red, tb, ring, xd, sv, tv, total;
};

// Compact tabu state of the wide streamed kernel: moves of the last TABU_RING iterations
// (one int each: key u << 9 | v, tenure << 18), so tenures up to TABU_RING - 1.
constexpr int TABU_RING = 1024;

// dglobal: D and D^T are read from global memory (the streamed kernels), not staged;
// gglobal: the wide streamed kernel (n above WIDE_N), which keeps no G and G^T: it reads
// F and F^T in global memory through the permutation.
__host__ __device__ inline Smem smem_plan(int n, int np, int lanes, int sym, bool dglobal = false,
                                          bool gglobal = false) {
    const int rs = row_stride(n);
    Smem s;
    int o = 0;
    auto take = [&o](int bytes) { int at = o; o += (bytes + 15) & ~15; return at; };
    // Matrices start 0, 64, 128, 192 bytes past a 256-byte boundary (G, G^T, D, D^T): the
    // lanes of one index read the same row of the four matrices at once, and 256 bytes
    // span every LDS bank, so equal skews would put all four reads in the same banks.
    auto take_mat = [&o](int skew) { o = ((o + 255) & ~255) + skew; return o; };
    if (dglobal) {
        s.d = s.dt = -1;
    } else {
        s.d = take_mat(128); o += n * rs;
        s.dt = sym ? s.d : take_mat(192); if (!sym) o += n * rs;
    }
    if (gglobal) {
        s.g = s.gt = -1;
    } else {
        s.g = take_mat(0); o += n * rs;
        s.gt = sym ? s.g : take_mat(64); if (!sym) o += n * rs;
    }
    s.acbe = take(np * 8);
    s.rpr = take(np * 4);
    s.rps = take(np * 4);
    s.kc = take(4 * 4);
    s.perm = take(np * 4);
    s.bestp = take(np * 4);
    s.pinv = take(np * 4);
    s.ten = take(lanes * 4);
    s.red = take(16 * 8);
    // (gglobal) compact tabu state: a bit per slot, one word per 8 x 4 tile position of
    // the padded grid, and the ring of recent moves
    s.tb = s.ring = s.xd = s.sv = -1;
    if (gglobal) {
        s.tb = take((np / 8) * (np / TILE_COLS) * 4);
        s.ring = take(TABU_RING * 4);
        // the permuted side rows of the row recomputation, two per family, RS bytes each
        s.sv = take(families(sym) * 2 * rs);
    }
    // (streamed kernels) the two row dot products of every (index, family) task, made by
    // whole waves; below WIDE_N also the side rows r and s of D and D^T, staged for them,
    // and RD_u, CD_u (ints) and d_uu (bytes) of every index (at n = 256 not symmetric the
    // plan takes 160 272 bytes, and the kernels' static LDS, at most 9.6 KB, the rest)
    s.tv = -1;
    if (dglobal) s.xd = take(families(sym) * np * 8);
    if (dglobal && !gglobal) {
        s.sv = take((sym ? 2 : 4) * rs);
        s.tv = take(2 * np * 4 + np);
    }
    s.total = o;
    return s;
}


// Arguments of the cost and neighbourhood-table kernels.
struct TableArgs {
    const uint8_t *mats;     // global [F | F^T | D | D^T], n rows of RS bytes each
    const int32_t *perms;    // [k][n]
    int64_t *costs;          // [k] or null
    int32_t *table;          // [k][m] or null
    int n, m, k;
    int sym;                 // F and D both symmetric
};

// Arguments of the search kernels (2opt and tabu).
struct SearchArgs {
    const uint8_t *mats;     // global [F | F^T | D | D^T]
    const int32_t *table;    // [k][m] neighbourhood of each start
    const int32_t *perms_in; // [k][n]
    int32_t *perm_out;       // [k][n]; may alias perms_in
    int64_t *cost_out;       // [k]
    int32_t *steps_out;      // [k] or null
    const int32_t *tiles;    // [ntiles] lane -> tile, g | b << 16, interior tiles first
    int n, m, ntiles, ninterior;
    int iters;               // tabu: iterations; 2opt: move cap (<= 0: none)
    int lo, hi;
    unsigned long long seed;
    long long start_base;
    int sym;
    int job0;                // search index of block 0
    int4 *tile_work;         // streamed kernels: per search, tile_stride int4 of tile state
    long long tile_stride;
    int32_t *freq;           // tabu: [k][m] exchange counts per search, or null
    int div;                 // with freq: diversification patience (0: none)
    int attr;                // with freq: tabu attribute, 0 pairs of locations, 1 units, 2 unit-locations
    int32_t *uloc;           // attr 2: [k][n][n] per search, until when a unit may not return to a location
    long long *trace;        // with freq: [k][trace_cap][4] (r, s, delta, cost after) per move, or null
    int trace_cap;
};

// With QAP_VERBOSE set in the environment, report a failed HIP call on stderr.
inline hipError_t report(hipError_t e, const char *what) {
    if (e != hipSuccess && std::getenv("QAP_VERBOSE"))
        std::fprintf(stderr, "libqap: %s: %s (%d)\n", what, hipGetErrorString(e), (int)e);
    return e;
}

// Largest dynamic LDS allocation a workgroup may request on the current device.
inline size_t max_dyn_smem() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 64 * 1024;
    return (size_t)v;
}

// Saved state of a search run in chunks of iterations (serving).  The arrays it
// refers to live beside it in device memory: the current and the best permutation (n
// each) and, in packed move order, the deltas of the current permutation and the
// iteration at which each move becomes free again (m each).
struct SearchState {
    long long cur, best;
    int it;      // next iteration to run, 1-based; 1 = not started
    int done;    // 1 once the last iteration ran or no move was allowed
    int moves;   // moves made so far
    int last_imp;   // with the frequency memory: the iteration of the last new best or diversification
};

// One search as the search kernels see it.
struct Item {
    const uint8_t *mats;      // global [F | F^T | D | D^T] of the instance
    const int32_t *tiles;     // lane -> tile for the item's tile shape
    const int32_t *table;     // neighbourhood of the start (read when the search starts)
    const int32_t *perm_in;   // start permutation
    int32_t *perm_out;        // best (tabu) or final (2opt) permutation, written when finished
    int64_t *cost_out;        // its cost
    int32_t *steps_out;       // moves made, or null
    SearchState *st;          // null: run from the start to `iters` in one go
    int32_t *st_perm, *st_bestp;
    int2 *st_du;              // chunked runs: (delta, tabu until) per packed pair index
    int n, m, sym, ntiles, ninterior, rows;
    int iters;                // tabu: last iteration of this run; 2opt: move cap (<= 0: none)
    int lo, hi;
    unsigned long long seed;
    long long start_id;
    // batched launches: offsets of this item's start / result / neighbourhood in the
    // launch's buffers (the pointers above are filled from them on the device)
    long long perm_off, out_off, table_off;
    // chunked runs (st != null): stop after about this many ticks of the device's
    // constant-rate clock, at an iteration boundary; 0 = run to `iters`
    long long budget;
    // streamed kernels: the search's tiles in global memory, pass-major, one int4 per
    // (pass, tile row, lane): deltas and tabu-until values (kept between chunks)
    int4 *tile_d, *tile_u;
    int stream;               // 1: the streamed kernel (tiles of STREAM_ROWS rows)
    long long tile_off;       // batched launches: offset of tile_d in the launch's tile work
    // tabu: the frequency memory, m counts of how often each pair of locations was
    // exchanged (packed pair index), zeroed when the search starts; null: not kept
    int32_t *freq;
    // with freq: after more than div iterations without a new
    // best, the next move is the least exchanged non-tabu pair; 0: never
    int div;
    // with freq: what is tabu, 0 the pair of locations exchanged, 1 the two units moved
    // (a move is tabu while either unit it would move is marked), 2 the return of a unit
    // to a location it left (a move is tabu when both units would return)
    int attr;
    int32_t *uloc;            // attr 2: [n][n], unit x location -> until when it may not return
    int32_t *st_mark;         // attr 1, chunked runs: the unit marks per location, kept between chunks
    // batched plans that keep the frequency memory: offsets of freq and uloc in the
    // plan's buffers (host side, while the plan is built)
    long long freq_off, uloc_off;
    // with freq: the first trace_cap moves as (r, s, delta, cost after), or null
    long long *trace;
    int trace_cap;
};

// The batched launch: one block per item of `items`; per-start buffers are shared by
// all items and addressed through the items' offsets.
struct BatchArgs {
    const Item *items;
    int count;
    int32_t *perms;    // starts in, best permutations out
    int64_t *best;
    int32_t *done;     // or null
    int32_t *table;    // neighbourhood of every start
    int4 *tile_work;   // tile state of the searches that run streamed
};

hipError_t launch_cost(const TableArgs &a, hipStream_t st);
hipError_t launch_table(const TableArgs &a, hipStream_t st);
// Neighbourhood tables of all items of a batch, one block per item.
hipError_t launch_table_batch(const BatchArgs &b, size_t smem, hipStream_t st);
size_t table_smem_bytes(int n);
// rows in {2, 4, 8, 16}; grid = number of searches in this launch; lanes = block size.
hipError_t launch_search(int rows, bool tabu, const SearchArgs &a, int grid, int lanes,
                         hipStream_t st);
size_t search_smem_bytes(int n, int rows, int lanes, int sym);
// Lanes of the persistent batched kernel, and whether a tile shape can serve n there.
constexpr int BATCH_LANES = 512;
int batch_shape_ok(int n, int rows, int ntiles, int sym);
// Kernel variants of the batched launch: register tiles of 2, 4, 8 rows and the streamed
// form on BATCH_LANES lanes, and for searches that need fewer lanes (a lane per tile and
// per (index, family) task) tiles of 2 rows on 128 or 256 lanes and of 4 rows on 256, so
// that more small searches share a compute unit; tiles of 4 rows also on 768 lanes (one
// task per lane, three waves per SIMD) for searches with more than BATCH_LANES tiles.
// One launch per variant.
// The wide streamed form (n above WIDE_N: G and G^T in global scratch, up to WIDE_MAXT
// tasks a lane) is the last variant.
enum { BV_R2 = 0, BV_R4, BV_R8, BV_STREAM, BV_R2_128, BV_R2_256, BV_R4_256, BV_R4_768, BV_WIDE, BV_COUNT };
// Whether a batched launch serves tile shape rows for this n (batch_shape_ok, or tiles of
// 4 rows on the 768-lane variant).
int batch_shape_ok_wide(int n, int rows, int ntiles, int sym);
// Variant of a batched search: rows 2, 4, 8 or the streamed form (the wide one above
// WIDE_N), ntiles tiles; -1 for a shape no batched kernel serves.
int batch_variant(int n, int rows, bool streamed, int ntiles, int sym);
// Lanes of a workgroup of that variant.
int batch_variant_lanes(int variant);
hipError_t launch_batch_group(int variant, const BatchArgs &b, size_t smem, hipStream_t st);
// Batched searches that keep the frequency memory (Item::freq, and Item::div, Item::attr,
// Item::uloc): one launch of BATCH_LANES lanes over items of tile rows 2, 4, 8 and the
// streamed form.
hipError_t launch_batch_freq(const BatchArgs &b, size_t smem, hipStream_t st);
// Static LDS of the kernels that run searches with the frequency memory for every tile
// shape (batch_freq_kernel, resume_freq_kernel): a plan's dynamic LDS must leave room
// for it (0 if the query fails).
size_t freq_static_lds();
int search_max_lanes(int rows);
// Workgroups of the register-tile search kernel for this shape that fit on one compute
// unit at once (HIP's occupancy query; 0 if it fails).
int search_blocks_per_cu(int n, int rows, bool tabu, int lanes, int sym);
// Streamed kernels (any n up to 256): tiles of STREAM_ROWS x 4 slots kept in global memory
// between passes, D read from global memory, BATCH_LANES lanes per search.  The wide form
// (n above WIDE_N, up to 512) keeps no G and G^T (it reads F and F^T through the
// permutation) and runs up to four (index, family) tasks per lane.
constexpr int STREAM_ROWS = 8;
constexpr int WIDE_MAXN = 512;
constexpr int WIDE_MAXT = 4 * WIDE_MAXN / BATCH_LANES;   // tasks a lane, n = 512 not symmetric
int stream_shape_ok(int n, int sym, size_t max_smem);
// int4 of tile state one streamed search needs (deltas, then tabu-until values)
__host__ __device__ inline long long stream_tile_int4(int ntiles) {
    const long long passes = (ntiles + BATCH_LANES - 1) / BATCH_LANES;
    return 2 * passes * STREAM_ROWS * BATCH_LANES;
}
size_t stream_smem_bytes(int n, int sym);
hipError_t launch_stream(bool tabu, const SearchArgs &a, int grid, hipStream_t st);
// Chunked runs of resumable searches: one block per item, pointers absolute.  Tables of
// items that start now (into their `table`), then one chunk of every item.
hipError_t launch_table_items(const Item *d_items, int count, size_t smem, hipStream_t st);
hipError_t launch_resume(const Item *d_items, int count, size_t smem, hipStream_t st);
// The same for items that keep the frequency memory (n up to WIDE_N).
hipError_t launch_resume_freq(const Item *d_items, int count, size_t smem, hipStream_t st);
// The same for items above WIDE_N (the wide streamed form).
hipError_t launch_resume_wide(const Item *d_items, int count, size_t smem, hipStream_t st);
// Lanes of a search workgroup for a tile shape, or 0 if the shape cannot serve n.
int search_lanes(int n, int rows, int ntiles, int sym);

}  // namespace qapk
