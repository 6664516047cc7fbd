// qap_api.hip -- host side of the C ABI declared in include/qap.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/qap.h"
#include "qap_host.h"
#include "qap_internal.h"

using namespace qapk;

namespace qaph {

const int kRowsChoices[kShapes] = {1, 2, 4, 8, 16};

struct TileSet {
    int32_t *d_tiles = nullptr;
    int ntiles = 0, ninterior = 0, lanes = 0;
};

// Tiles of `rows` x 4 that hold at least one move (u < v), interior tiles first, each
// group in row-major (g, b) order; a tile is interior when no row or column passes n.
std::vector<int32_t> enumerate_tiles(int n, int rows, int *ninterior) {
    std::vector<int32_t> inner, outer;
    const int ng = (n + rows - 1) / rows, nb = (n + TILE_COLS - 1) / TILE_COLS;
    for (int g = 0; g < ng; ++g)
        for (int b = 0; b < nb; ++b) {
            const int ulo = g * rows, vhi = std::min(TILE_COLS * b + TILE_COLS, n) - 1;
            if (ulo >= vhi) continue;
            const bool interior = g * rows + rows <= n && TILE_COLS * b + TILE_COLS <= n;
            (interior ? inner : outer).push_back(g | (b << 16));
        }
    *ninterior = (int)inner.size();
    inner.insert(inner.end(), outer.begin(), outer.end());
    return inner;
}

int pack_instance(const int32_t *F, const int32_t *D, int n, std::vector<uint8_t> &pack, int *sym) {
    bool symF = true, symD = true;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int32_t f = F[(size_t)i * n + j], d = D[(size_t)i * n + j];
            if (f < 0 || f > 255 || d < 0 || d > 255) return QAP_E_RANGE;
            if (f != F[(size_t)j * n + i]) symF = false;
            if (d != D[(size_t)j * n + i]) symD = false;
        }
    *sym = (symF && symD) ? 1 : 0;
    const int rs = row_stride(n);
    pack.assign((size_t)4 * n * rs, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            pack[(size_t)0 * n * rs + (size_t)i * rs + j] = (uint8_t)F[(size_t)i * n + j];
            pack[(size_t)1 * n * rs + (size_t)i * rs + j] = (uint8_t)F[(size_t)j * n + i];
            pack[(size_t)2 * n * rs + (size_t)i * rs + j] = (uint8_t)D[(size_t)i * n + j];
            pack[(size_t)3 * n * rs + (size_t)i * rs + j] = (uint8_t)D[(size_t)j * n + i];
        }
    return QAP_OK;
}

int dev_err_at(hipError_t e, const char *where) {
    if (e == hipSuccess) return QAP_OK;
    static const bool verbose = std::getenv("QAP_VERBOSE") != nullptr;
    if (verbose) std::fprintf(stderr, "libqap: %s: %s (%d)\n", where, hipGetErrorString(e), (int)e);
    return e == hipErrorOutOfMemory ? QAP_E_NOMEM : QAP_E_DEVICE;
}

// Side streams a batched launch forks into: one fewer than the hardware queues HIP gives
// the process (GPU_MAX_HW_QUEUES, 4 unless set), so that each lane has a queue of its own
// beside the caller's stream; QAP_BATCH_LANES overrides the count.
static int side_lanes() {
    auto env_int = [](const char *name, int dflt) {
        const char *v = std::getenv(name);
        return v && *v ? std::atoi(v) : dflt;
    };
    const int forced = env_int("QAP_BATCH_LANES", 0);
    const int lanes = forced > 0 ? forced : env_int("GPU_MAX_HW_QUEUES", 4) - 1;
    return std::max(1, std::min(lanes, (int)BV_COUNT));
}

bool check_perms(const int32_t *perms, int k, int n) {
    std::vector<int> seen(n);
    for (int j = 0; j < k; ++j) {
        std::fill(seen.begin(), seen.end(), 0);
        const int32_t *p = perms + (size_t)j * n;
        for (int i = 0; i < n; ++i) {
            if (p[i] < 0 || p[i] >= n || seen[p[i]]) return false;
            seen[p[i]] = 1;
        }
    }
    return true;
}

}  // namespace qaph

using namespace qaph;

struct qap_ctx {
    int n = 0, m = 0, sym = 0, device = 0;
    size_t max_smem = 0;
    uint8_t *d_mats = nullptr;       // [F | F^T | D | D^T] u8, n rows of row_stride(n) bytes
    TileSet tiles[kShapes];          // one per entry of kRowsChoices
    // per algorithm (0 tabu, 1 2opt, 2 batched tabu): index into kRowsChoices, kStream for
    // the streamed kernel, -1 when no kernel serves this n
    int rows_choice[3] = {0, 0, 0};
    int rows_default[3] = {0, 0, 0};
    // tabu and 2opt: the shape is picked per launch (launch_shape) until one is set
    int auto_rows[2] = {1, 1};
    int cus = 0;                     // compute units of the device
    int blocks_cache[2][kShapes];    // workgroups per compute unit per shape, -1 = not asked yet
    int stream_ok = 0;               // the streamed kernel serves this n
};

namespace qaph {
bool handle_view(const qap_ctx *h, const uint8_t **mats, int *n, int *sym, int *device) {
    if (!h) return false;
    *mats = h->d_mats;
    *n = h->n;
    *sym = h->sym;
    *device = h->device;
    return true;
}
}  // namespace qaph

namespace {

// Shape index of the streamed kernel (tiles of STREAM_ROWS rows in global memory); the
// ABI names it rows = -STREAM_ROWS.
constexpr int kStream = kShapes;
// The batched kernels serve rows 2, 4 and 8: shape indices kBatchFirst .. kBatchFirst + 2.
constexpr int kBatchFirst = 1;
// Shape index of the STREAM_ROWS tile list, which the streamed kernel walks.
constexpr int kStreamList = 3;

int rows_index(int rows) {
    if (rows == -STREAM_ROWS) return kStream;
    for (int i = 0; i < kShapes; ++i)
        if (kRowsChoices[i] == rows) return i;
    return -1;
}

int shape_rows(int ri) { return ri == kStream ? -STREAM_ROWS : kRowsChoices[ri]; }

// The tile list a shape uses (the streamed kernel uses the STREAM_ROWS list).
const TileSet &shape_tiles(const qap_ctx *h, int ri) { return h->tiles[ri == kStream ? kStreamList : ri]; }

bool shape_fits(const qap_ctx *h, int ri) {
    if (ri == kStream) return h->stream_ok != 0;
    if (ri < 0 || ri >= kShapes || h->n > WIDE_N) return false;
    const TileSet &ts = h->tiles[ri];
    if (ts.lanes < 64 || ts.lanes > search_max_lanes(kRowsChoices[ri])) return false;
    if (ts.ntiles > ts.lanes) return false;
    return search_smem_bytes(h->n, kRowsChoices[ri], ts.lanes, h->sym) <= h->max_smem;
}

// Default tile shape: the smallest tile that fits (the most lanes per search, hence the
// shortest dependency chain per iteration).
int default_rows(const qap_ctx *h) {
    for (int i = 0; i < kShapes; ++i)
        if (shape_fits(h, i)) return i;
    return h->stream_ok ? kStream : -1;
}

// Shape a launch of k tabu (algo 0) or 2opt (algo 1) searches uses: the handle's shape
// once one is set, else the fitting register shape that needs the fewest rounds of
// workgroups over the device's compute units, ties going to the smallest tile (the most
// lanes per search, hence the shortest dependency chain per iteration); the streamed
// kernel when no register shape fits.  A small tile is fastest while every search has a
// compute unit of its own; with many more searches than compute units a larger tile on
// fewer lanes lets more searches share a compute unit.
int launch_shape(qap_ctx *h, int algo, int k) {
    if (algo == 2 || !h->auto_rows[algo]) return h->rows_choice[algo];
    int best = -1;
    long long best_rounds = 0;
    for (int ri = 0; ri < kShapes; ++ri) {
        if (!shape_fits(h, ri)) continue;
        int &nb = h->blocks_cache[algo][ri];
        if (nb < 0) nb = search_blocks_per_cu(h->n, kRowsChoices[ri], algo == 0, h->tiles[ri].lanes, h->sym);
        if (nb <= 0 || h->cus <= 0) continue;
        const long long per_round = (long long)nb * h->cus;
        const long long rounds = ((long long)k + per_round - 1) / per_round;
        if (best < 0 || rounds < best_rounds) {
            best = ri;
            best_rounds = rounds;
        }
    }
    return best >= 0 ? best : h->rows_choice[algo];
}


// RAII device buffer for the blocking entry points.
struct DevBuf {
    void *p = nullptr;
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// Private stream of a blocking entry point.
struct HostCall {
    hipStream_t st = nullptr;
    ~HostCall() { if (st) (void)hipStreamDestroy(st); }
    hipError_t init() { return hipStreamCreateWithFlags(&st, hipStreamNonBlocking); }
};

// Arguments shared by every search of a launch with tile shape ri (its tile list).
SearchArgs base_args(const qap_ctx *h, int ri) {
    const TileSet &ts = shape_tiles(h, ri);
    SearchArgs a{};
    a.mats = h->d_mats;
    a.n = h->n;
    a.m = h->m;
    a.tiles = ts.d_tiles;
    a.ntiles = ts.ntiles;
    a.ninterior = ts.ninterior;
    a.sym = h->sym;
    return a;
}

// Neighbourhood tables for the starts, in stream-ordered scratch memory.
int make_tables(qap_ctx *h, const int32_t *d_perms, int k, int32_t **d_table, hipStream_t st) {
    hipError_t e = report(hipMallocAsync((void **)d_table, (size_t)k * h->m * sizeof(int32_t) + 16, st),
                          "hipMallocAsync");
    if (e != hipSuccess) return dev_err(e);
    TableArgs ta{h->d_mats, d_perms, nullptr, *d_table, h->n, h->m, k, h->sym};
    e = launch_table(ta, st);
    if (e != hipSuccess) { (void)hipFreeAsync(*d_table, st); return dev_err(e); }
    return QAP_OK;
}

// Scratch buffer of the streamed kernels supplied by the caller (the entry point that
// allocates nothing): tile state of every search of the launch.
struct StreamScratch {
    int4 *tile_work;
};

hipError_t launch_shaped(qap_ctx *h, int algo, int ri, SearchArgs a, int k, hipStream_t st, bool plain,
                         const StreamScratch *pre = nullptr);

hipError_t launch_searches(qap_ctx *h, int algo, int32_t *d_perms, const int32_t *d_table, int k, int iters,
                           int lo, int hi, uint64_t seed, int64_t start_base, int64_t *d_cost, int32_t *d_steps,
                           hipStream_t st, bool plain, int32_t *d_freq = nullptr, int div = 0, int attr = 0,
                           int ri = -1, const StreamScratch *pre = nullptr, long long *d_trace = nullptr,
                           int trace_cap = 0) {
    // one shape for the whole launch: its kernel and its tile list
    if (ri < 0) ri = launch_shape(h, algo, k);
    if (ri < 0) return hipErrorInvalidValue;
    SearchArgs a = base_args(h, ri);
    a.table = d_table;
    a.perms_in = d_perms;
    a.perm_out = d_perms;
    a.cost_out = d_cost;
    a.steps_out = d_steps;
    a.iters = iters;
    a.lo = lo;
    a.hi = hi;
    a.seed = seed;
    a.start_base = start_base;
    a.freq = d_freq;
    a.div = div;
    a.attr = attr;
    a.trace = d_trace;
    a.trace_cap = trace_cap;
    hipError_t e = hipSuccess;
    if (d_freq && attr == 2) {
        // the unit-location table of every search, in stream-ordered scratch
        e = report(hipMallocAsync((void **)&a.uloc, (size_t)k * h->n * h->n * sizeof(int32_t) + 16, st),
                   "hipMallocAsync");
        if (e != hipSuccess) return e;
        e = launch_shaped(h, algo, ri, a, k, st, plain);
        const hipError_t e2 = hipFreeAsync(a.uloc, st);
        return e != hipSuccess ? e : e2;
    }
    return launch_shaped(h, algo, ri, a, k, st, plain, pre);
}

// The launches of one search call with tile shape ri (the streamed kernel takes its tile
// state from stream-ordered scratch, or from `pre`).
hipError_t launch_shaped(qap_ctx *h, int algo, int ri, SearchArgs a, int k, hipStream_t st, bool plain,
                         const StreamScratch *pre) {
    hipError_t e = hipSuccess;
    if (ri == kStream && pre) {
        a.tile_stride = stream_tile_int4(a.ntiles);
        a.tile_work = pre->tile_work;
        a.job0 = 0;
        return launch_stream(algo == 0, a, k, st);
    }
    if (ri == kStream) {
        // tile state in stream-ordered scratch, one slice per search of a launch
        a.tile_stride = stream_tile_int4(a.ntiles);
        const int per_launch = plain ? 1 : k;
        e = report(hipMallocAsync((void **)&a.tile_work, (size_t)per_launch * a.tile_stride * sizeof(int4), st),
                   "hipMallocAsync");
        if (e != hipSuccess) return e;
        if (plain) {
            for (int j = 0; j < k && e == hipSuccess; ++j) {
                a.job0 = j;
                e = launch_stream(algo == 0, a, 1, st);
            }
        } else {
            a.job0 = 0;
            e = launch_stream(algo == 0, a, k, st);
        }
        const hipError_t e2 = hipFreeAsync(a.tile_work, st);
        return e != hipSuccess ? e : e2;
    }
    const int rows = kRowsChoices[ri];
    const int lanes = h->tiles[ri].lanes;
    if (plain) {
        for (int j = 0; j < k && e == hipSuccess; ++j) {
            a.job0 = j;
            e = launch_search(rows, algo == 0, a, 1, lanes, st);
        }
    } else {
        a.job0 = 0;
        e = launch_search(rows, algo == 0, a, k, lanes, st);
    }
    return e;
}

int run_search(qap_ctx *h, int algo, int32_t *d_perms, int k, int iters, int lo, int hi, uint64_t seed,
               int64_t start_base, int64_t *d_cost, int32_t *d_steps, hipStream_t st, bool plain,
               int32_t *d_freq = nullptr, int div = 0, int attr = 0, long long *d_trace = nullptr,
               int trace_cap = 0) {
    if (h->rows_choice[algo] < 0) return QAP_E_UNSUPPORTED;
    if (k == 0) return QAP_OK;
    int32_t *d_table = nullptr;
    int rc = make_tables(h, d_perms, k, &d_table, st);
    if (rc != QAP_OK) return rc;
    hipError_t e = launch_searches(h, algo, d_perms, d_table, k, iters, lo, hi, seed, start_base, d_cost,
                                   d_steps, st, plain, d_freq, div, attr, -1, nullptr, d_trace, trace_cap);
    hipError_t e2 = hipFreeAsync(d_table, st);
    if (e == hipSuccess) e = e2;
    return dev_err(e);
}

// Whether tile shape ri serves this instance in the batched kernel (fixed workgroup of
// BATCH_LANES lanes, rows 2, 4 or 8).
bool batch_fits(const qap_ctx *h, int ri) {
    if (ri == kStream) return h->stream_ok != 0;   // above WIDE_N, the wide streamed form
    if (h->n > WIDE_N) return false;
    if (ri < kBatchFirst || ri > kBatchFirst + 2) return false;
    const TileSet &ts = h->tiles[ri];
    const int rows = kRowsChoices[ri];
    const int var = batch_variant(h->n, rows, false, ts.ntiles, h->sym);
    if (var < 0) return false;   // no batched kernel for this shape
    const int lanes = batch_variant_lanes(var);
    return ts.d_tiles && batch_shape_ok_wide(h->n, rows, ts.ntiles, h->sym) &&
           search_smem_bytes(h->n, rows, lanes, h->sym) <= h->max_smem;
}

// Default batched shape: the smallest tile that fits.
int batch_default(const qap_ctx *h) {
    for (int i = kBatchFirst; i < kBatchFirst + 3; ++i)
        if (batch_fits(h, i)) return i;
    return h->stream_ok ? kStream : -1;
}

bool algo_fits(const qap_ctx *h, int algo, int ri) { return algo == 2 ? batch_fits(h, ri) : shape_fits(h, ri); }

// Tile shape of an instance in the batched kernel: the handle's choice for algo 2.
int batch_shape(const qap_ctx *h) {
    const int ri = h->rows_choice[2];
    return ri >= 0 && batch_fits(h, ri) ? ri : -1;
}

// Starts for timing runs: fixed pseudo-random permutations (splitmix64 driving a
// Fisher-Yates shuffle), so that every shape is timed on the same work.
void timing_starts(int n, int k, std::vector<int32_t> &p) {
    p.resize((size_t)k * n);
    uint64_t x = 0x243F6A8885A308D3ull;
    for (int j = 0; j < k; ++j) {
        int32_t *q = p.data() + (size_t)j * n;
        for (int i = 0; i < n; ++i) q[i] = i;
        for (int i = n - 1; i > 0; --i) {
            uint64_t z = (x += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            std::swap(q[i], q[z % (uint64_t)(i + 1)]);
        }
    }
}

}  // namespace

// Starting neighbourhoods of one instance above WIDE_N in a batch: its k starts and
// tables are contiguous at these offsets of the run's starts and the plan's tables.
struct WideTable {
    const uint8_t *mats;
    int n, m, k, sym;
    long long perm_off, table_off;
};

struct qap_batch {
    int count = 0;                  // searches (items)
    long long perm_ints = 0, table_ints = 0, tile_int4 = 0;
    Item *d_items = nullptr;
    int32_t *d_table = nullptr;
    int4 *d_tile_work = nullptr;    // tile state of the streamed searches
    size_t table_smem = 0;
    // starting neighbourhoods of instances above WIDE_N: one Eq. (2) launch per instance
    // (offsets into the run's starts and the plan's tables); the matrix-core table kernel
    // takes every other item
    std::vector<WideTable> wide_tables;
    // items are grouped by kernel variant (tile shape); one launch per non-empty group
    int group_begin[BV_COUNT] = {}, group_count[BV_COUNT] = {};
    size_t group_smem[BV_COUNT] = {};
    // The groups run on `nlanes` side streams forked from the caller's stream, the groups
    // of one lane back to back: lane_groups[lane_begin[l] .. lane_begin[l + 1]).  Streams
    // beyond the device's hardware queues would share queues, and kernels on one queue
    // run in order, so there are at most as many lanes as free queues; the groups are
    // dealt to them by estimated work, largest first, each to the least loaded lane.
    int nlanes = 0;
    int lane_begin[BV_COUNT + 1] = {};
    int lane_groups[BV_COUNT] = {};
    hipStream_t side[BV_COUNT] = {};
    hipEvent_t ev_fork = nullptr, ev_join[BV_COUNT] = {};
    // plans made by qap_batch_create_freq: every search keeps its frequency memory (and may
    // diversify or use a unit attribute); all run in one launch of batch_freq_kernel
    bool freq_mode = false;
    size_t freq_smem = 0;
    long long freq_ints = 0;        // counts of every search, instance order, start order
    int32_t *d_freq = nullptr;
    int32_t *d_uloc = nullptr;      // attr 2: unit x location table of every such search
};

namespace {

int item_variant(const Item &it) { return batch_variant(it.n, it.rows, it.stream != 0, it.ntiles, it.sym); }

// ---- fixed scratch of qap_tabu_noalloc_async: one array per GPU, held until the process
//      ends.  Host code never passes the array's name to a kernel (on the host it only
//      names the symbol); the device address of each GPU's copy is looked up once, with
//      that GPU current, and kept in noalloc_ptr.
__device__ __align__(256) unsigned char scratch[QAP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
unsigned char *noalloc_ptr[kMaxDevices] = {};

// Look up this device's copy of `scratch` (the current device); QAP_OK once known.
int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return QAP_E_DEVICE;
    std::lock_guard<std::mutex> g(noalloc_mu);
    if (noalloc_ptr[device]) return QAP_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return dev_err(e != hipSuccess ? e : hipErrorInvalidSymbol);
    noalloc_ptr[device] = static_cast<unsigned char *>(ptr);
    return QAP_OK;
}

unsigned char *noalloc_base(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(noalloc_mu);
    return noalloc_ptr[device];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

const char *qap_strerror(int code) {
    switch (code) {
        case QAP_OK: return "ok";
        case QAP_E_INVALID: return "invalid argument";
        case QAP_E_NOT_PERM: return "a row is not a permutation of 0..n-1";
        case QAP_E_RANGE: return "a flow or distance lies outside [0, 255]";
        case QAP_E_DEVICE: return "HIP device error";
        case QAP_E_NOMEM: return "out of memory";
        case QAP_E_BUSY: return "server queue full";
        case QAP_E_UNSUPPORTED: return "unsupported by this build";
        case QAP_E_SCRATCH: return "the call needs more than the fixed scratch of qap_tabu_noalloc_async";
        default: return "unknown error";
    }
}

int qap_create(const int32_t *F, const int32_t *D, int32_t n, qap_handle *out) {
    if (!F || !D || !out || n < 2 || n > QAP_NMAX) return QAP_E_INVALID;
    *out = nullptr;
    std::vector<uint8_t> pack;
    int sym = 0;
    const int prc = pack_instance(F, D, n, pack, &sym);
    if (prc != QAP_OK) return prc;
    qap_ctx *h = new (std::nothrow) qap_ctx;
    if (!h) return QAP_E_NOMEM;
    h->n = n;
    h->m = n * (n - 1) / 2;
    h->sym = sym;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return QAP_E_DEVICE; }
    int smem = 0;
    if (hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess) {
        delete h;
        return QAP_E_DEVICE;
    }
    h->max_smem = (size_t)smem;
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        delete h;
        return QAP_E_DEVICE;
    }
    for (auto &row : h->blocks_cache)
        for (int &x : row) x = -1;
    hipError_t e = hipMalloc((void **)&h->d_mats, pack.size());
    if (e == hipSuccess) e = hipMemcpy(h->d_mats, pack.data(), pack.size(), hipMemcpyHostToDevice);
    for (int i = 0; i < kShapes && e == hipSuccess; ++i) {
        int ninner = 0;
        std::vector<int32_t> tl = enumerate_tiles(n, kRowsChoices[i], &ninner);
        TileSet &ts = h->tiles[i];
        ts.ntiles = (int)tl.size();
        ts.ninterior = ninner;
        ts.lanes = search_lanes(n, kRowsChoices[i], ts.ntiles, h->sym);
        e = hipMalloc((void **)&ts.d_tiles, tl.size() * sizeof(int32_t) + 16);
        if (e == hipSuccess)
            e = hipMemcpy(ts.d_tiles, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        qap_destroy(h);
        return dev_err(e);
    }
    // once per device, with it current: the address of its fixed scratch array
    const int src = noalloc_setup(h->device);
    if (src != QAP_OK) {
        qap_destroy(h);
        return src;
    }
    h->stream_ok = stream_shape_ok(n, h->sym, h->max_smem);
    const int d = default_rows(h);   // -1: no search kernel shape fits this n
    h->rows_default[0] = h->rows_default[1] = d;
    h->rows_choice[0] = h->rows_choice[1] = d;
    h->rows_default[2] = h->rows_choice[2] = batch_default(h);
    *out = h;
    return QAP_OK;
}

int qap_destroy(qap_handle h) {
    if (!h) return QAP_OK;
    if (h->d_mats) (void)hipFree(h->d_mats);
    for (auto &ts : h->tiles)
        if (ts.d_tiles) (void)hipFree(ts.d_tiles);
    delete h;
    return QAP_OK;
}

int qap_size(qap_handle h) { return h ? h->n : QAP_E_INVALID; }

int qap_set_tile_rows(qap_handle h, int32_t algo, int32_t rows) {
    if (!h || algo < 0 || algo > 2) return QAP_E_INVALID;
    if (rows == 0) {
        h->rows_choice[algo] = h->rows_default[algo];
        if (algo < 2) h->auto_rows[algo] = 1;
        return QAP_OK;
    }
    const int ri = rows_index(rows);
    if (ri < 0) return QAP_E_INVALID;
    if (!algo_fits(h, algo, ri)) return QAP_E_UNSUPPORTED;
    h->rows_choice[algo] = ri;
    if (algo < 2) h->auto_rows[algo] = 0;
    return QAP_OK;
}

int qap_get_tile_rows(qap_handle h, int32_t algo, int32_t *lanes_out) {
    return qap_launch_tile_rows(h, algo, 1, lanes_out);
}

int qap_launch_tile_rows(qap_handle h, int32_t algo, int32_t k, int32_t *lanes_out) {
    if (!h || algo < 0 || algo > 2 || k < 1) return QAP_E_INVALID;
    if (h->rows_choice[algo] < 0) return QAP_E_UNSUPPORTED;
    const int ri = launch_shape(h, algo, k);
    if (lanes_out) {
        if (ri == kStream)
            *lanes_out = BATCH_LANES;
        else if (algo == 2)   // the batched workgroup this instance's searches get
            *lanes_out = batch_variant_lanes(batch_variant(h->n, kRowsChoices[ri], false, h->tiles[ri].ntiles, h->sym));
        else
            *lanes_out = h->tiles[ri].lanes;
    }
    return shape_rows(ri);
}

int qap_tune_tile_rows(qap_handle h, int32_t algo, int32_t k, int32_t iters, float *ms_out) {
    if (!h || algo < 0 || algo > 2 || k <= 0 || iters <= 0) return QAP_E_INVALID;
    for (int i = 0; i <= kStream; ++i)
        if (ms_out) ms_out[i] = -1.0f;
    const int n = h->n;
    std::vector<int32_t> hp;
    timing_starts(n, k, hp);
    const int lo = std::max(0, n * 9 / 10), hi = n + n / 10;
    HostCall c;
    DevBuf ds, dw, db, dd, dt;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = c.init();
    if (e == hipSuccess) e = ds.alloc(hp.size() * 4);
    if (e == hipSuccess) e = dw.alloc(hp.size() * 4);
    if (e == hipSuccess) e = db.alloc((size_t)k * 8);
    if (e == hipSuccess) e = dd.alloc((size_t)k * 4);
    if (e == hipSuccess && algo < 2) e = dt.alloc((size_t)k * h->m * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(ds.p, hp.data(), hp.size() * 4, hipMemcpyHostToDevice, c.st);
    const int saved = h->rows_choice[algo];
    const int saved_auto = algo < 2 ? h->auto_rows[algo] : 0;
    if (algo < 2) h->auto_rows[algo] = 0;   // time exactly the shape set below
    int best = -1, rc = QAP_OK;
    float best_ms = 0.0f;
    for (int ri = 0; ri <= kStream && e == hipSuccess && rc == QAP_OK; ++ri) {
        if (!algo_fits(h, algo, ri)) continue;
        qap_batch_handle b = nullptr;
        if (algo == 2) {
            const int32_t rows = shape_rows(ri);
            const uint64_t seed = 1;
            const qap_handle hh = h;
            rc = qap_batch_create(&hh, 1, &k, iters, &lo, &hi, &seed, &rows, &b);
            if (rc != QAP_OK) break;
        }
        h->rows_choice[algo] = ri;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first run warms up
            e = hipMemcpyAsync(dw.p, ds.p, hp.size() * 4, hipMemcpyDeviceToDevice, c.st);
            int32_t *w = (int32_t *)dw.p;
            if (e == hipSuccess && algo < 2) {
                TableArgs ta{h->d_mats, w, nullptr, (int32_t *)dt.p, n, h->m, k, h->sym};
                e = launch_table(ta, c.st);
            } else if (e == hipSuccess) {
                rc = qap_batch_tables_async(b, w, c.st);
            }
            if (e == hipSuccess && rc == QAP_OK) e = hipEventRecord(e0, c.st);
            if (e == hipSuccess && rc == QAP_OK) {
                if (algo < 2)
                    e = launch_searches(h, algo, w, (const int32_t *)dt.p, k, iters, lo, hi, 1, 0, (int64_t *)db.p,
                                        (int32_t *)dd.p, c.st, false);
                else
                    rc = qap_batch_search_async(b, w, (int64_t *)db.p, (int32_t *)dd.p, c.st);
            }
            if (e == hipSuccess && rc == QAP_OK) e = hipEventRecord(e1, c.st);
            if (e == hipSuccess && rc == QAP_OK) e = hipEventSynchronize(e1);
            if (e == hipSuccess && rc == QAP_OK) e = hipEventElapsedTime(&ms, e0, e1);
        }
        qap_batch_destroy(b);
        if (e != hipSuccess || rc != QAP_OK) break;
        if (ms_out) ms_out[ri] = ms;
        if (best < 0 || ms < best_ms) {
            best = ri;
            best_ms = ms;
        }
    }
    h->rows_choice[algo] = best >= 0 ? best : saved;
    if (algo < 2 && best < 0) h->auto_rows[algo] = saved_auto;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_err(e);
    if (rc != QAP_OK) return rc;
    return best >= 0 ? shape_rows(best) : QAP_E_UNSUPPORTED;
}

int qap_cost_async(qap_handle h, const int32_t *d_perms, int32_t k, int64_t *d_costs, void *stream) {
    if (!h || k < 0 || (k > 0 && (!d_perms || !d_costs))) return QAP_E_INVALID;
    TableArgs a{h->d_mats, d_perms, d_costs, nullptr, h->n, h->m, k, h->sym};
    return dev_err(launch_cost(a, (hipStream_t)stream));
}

int qap_delta_table_async(qap_handle h, const int32_t *d_perms, int32_t k, int32_t *d_table, void *stream) {
    if (!h || k < 0 || (k > 0 && (!d_perms || !d_table))) return QAP_E_INVALID;
    TableArgs a{h->d_mats, d_perms, nullptr, d_table, h->n, h->m, k, h->sym};
    return dev_err(launch_table(a, (hipStream_t)stream));
}

int qap_2opt_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t max_iters, int64_t *d_costs,
                   int32_t *d_steps, void *stream) {
    if (!h || k < 0 || (k > 0 && (!d_perms || !d_costs))) return QAP_E_INVALID;
    return run_search(h, 1, d_perms, k, max_iters, 0, 0, 0, 0, d_costs, d_steps, (hipStream_t)stream, false);
}

static int tabu_args_ok(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                        int64_t *d_best) {
    return h && k >= 0 && tenure_args_ok(iters, lo, hi) && (k == 0 || (d_perms && d_best));
}

int qap_tabu_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                   uint64_t seed, int64_t start_base, int64_t *d_best, int32_t *d_done, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best)) return QAP_E_INVALID;
    return run_search(h, 0, d_perms, k, iters, lo, hi, seed, start_base, d_best, d_done, (hipStream_t)stream,
                      false);
}

int qap_tabu_freq_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                        uint64_t seed, int64_t start_base, int32_t div, int32_t attr, int64_t *d_best,
                        int32_t *d_done, int32_t *d_freq, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best) || (k > 0 && !d_freq) || div < 0 || attr < 0 ||
        attr > 2)
        return QAP_E_INVALID;
    return run_search(h, 0, d_perms, k, iters, lo, hi, seed, start_base, d_best, d_done, (hipStream_t)stream,
                      false, d_freq, div, attr);
}

int qap_tabu_trace_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                         uint64_t seed, int64_t start_base, int32_t div, int32_t attr, int64_t *d_best,
                         int32_t *d_done, int32_t *d_freq, int64_t *d_trace, int32_t trace_cap, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best) || (k > 0 && (!d_freq || !d_trace)) || div < 0 ||
        attr < 0 || attr > 2 || trace_cap < 0)
        return QAP_E_INVALID;
    return run_search(h, 0, d_perms, k, iters, lo, hi, seed, start_base, d_best, d_done, (hipStream_t)stream,
                      false, d_freq, div, attr, reinterpret_cast<long long *>(d_trace), trace_cap);
}

int qap_tabu_plain_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                         uint64_t seed, int64_t start_base, int64_t *d_best, int32_t *d_done, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best)) return QAP_E_INVALID;
    return run_search(h, 0, d_perms, k, iters, lo, hi, seed, start_base, d_best, d_done, (hipStream_t)stream,
                      true);
}

int qap_2opt_with_table_async(qap_handle h, int32_t *d_perms, const int32_t *d_table, int32_t k,
                              int32_t max_iters, int64_t *d_costs, int32_t *d_steps, void *stream) {
    if (!h || k < 0 || (k > 0 && (!d_perms || !d_costs || !d_table))) return QAP_E_INVALID;
    if (h->rows_choice[1] < 0) return QAP_E_UNSUPPORTED;
    if (k == 0) return QAP_OK;
    return dev_err(launch_searches(h, 1, d_perms, d_table, k, max_iters, 0, 0, 0, 0, d_costs, d_steps,
                                   (hipStream_t)stream, false));
}

int qap_tabu_with_table_async(qap_handle h, int32_t *d_perms, const int32_t *d_table, int32_t k,
                              int32_t iters, int32_t lo, int32_t hi, uint64_t seed, int64_t start_base,
                              int64_t *d_best, int32_t *d_done, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best) || (k > 0 && !d_table)) return QAP_E_INVALID;
    if (h->rows_choice[0] < 0) return QAP_E_UNSUPPORTED;
    if (k == 0) return QAP_OK;
    return dev_err(launch_searches(h, 0, d_perms, d_table, k, iters, lo, hi, seed, start_base, d_best, d_done,
                                   (hipStream_t)stream, false));
}

int qap_tabu_noalloc_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
                           uint64_t seed, int64_t start_base, int64_t *d_best, int32_t *d_done, void *stream) {
    if (!tabu_args_ok(h, d_perms, k, iters, lo, hi, d_best)) return QAP_E_INVALID;
    if (h->rows_choice[0] < 0) return QAP_E_UNSUPPORTED;
    if (k == 0) return QAP_OK;
    unsigned char *base = noalloc_base(h->device);
    if (!base) return QAP_E_DEVICE;
    // the shape of this launch decides what it needs beside the tables
    const int ri = launch_shape(h, 0, k);
    if (ri < 0) return QAP_E_UNSUPPORTED;
    const size_t table_bytes = align256((size_t)k * h->m * sizeof(int32_t));
    size_t tile_bytes = 0;
    if (ri == kStream)
        tile_bytes = align256((size_t)k * stream_tile_int4(shape_tiles(h, ri).ntiles) * sizeof(int4));
    if (table_bytes + tile_bytes > (size_t)QAP_NOALLOC_SCRATCH_BYTES) return QAP_E_SCRATCH;
    // every byte used is written before it is read (tables by the table kernel, tile state
    // when each search starts), so nothing needs clearing
    int32_t *d_table = reinterpret_cast<int32_t *>(base);
    StreamScratch pre{reinterpret_cast<int4 *>(base + table_bytes)};
    const hipStream_t st = (hipStream_t)stream;
    TableArgs ta{h->d_mats, d_perms, nullptr, d_table, h->n, h->m, k, h->sym};
    hipError_t e = launch_table(ta, st);
    if (e == hipSuccess)
        e = launch_searches(h, 0, d_perms, d_table, k, iters, lo, hi, seed, start_base, d_best, d_done, st, false,
                            nullptr, 0, 0, ri, &pre);
    return dev_err(e);
}

// ---- blocking host entry points: validate, copy in, run on a private stream, copy out


int qap_cost(qap_handle h, const int32_t *perms, int32_t k, int64_t *costs) {
    if (!h || k < 0 || (k > 0 && (!perms || !costs))) return QAP_E_INVALID;
    if (!check_perms(perms, k, h->n)) return QAP_E_NOT_PERM;
    if (k == 0) return QAP_OK;
    HostCall c;
    DevBuf dp, dc;
    hipError_t e = c.init();
    if (e == hipSuccess) e = dp.alloc((size_t)k * h->n * 4);
    if (e == hipSuccess) e = dc.alloc((size_t)k * 8);
    if (e == hipSuccess) e = hipMemcpyAsync(dp.p, perms, (size_t)k * h->n * 4, hipMemcpyHostToDevice, c.st);
    if (e != hipSuccess) return dev_err(e);
    int rc = qap_cost_async(h, (const int32_t *)dp.p, k, (int64_t *)dc.p, c.st);
    if (rc != QAP_OK) return rc;
    e = hipMemcpyAsync(costs, dc.p, (size_t)k * 8, hipMemcpyDeviceToHost, c.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    return dev_err(e);
}

int qap_delta_table(qap_handle h, const int32_t *perms, int32_t k, int32_t *table) {
    if (!h || k < 0 || (k > 0 && (!perms || !table))) return QAP_E_INVALID;
    if (!check_perms(perms, k, h->n)) return QAP_E_NOT_PERM;
    if (k == 0) return QAP_OK;
    HostCall c;
    DevBuf dp, dt;
    const size_t tb = (size_t)k * h->m * 4;
    hipError_t e = c.init();
    if (e == hipSuccess) e = dp.alloc((size_t)k * h->n * 4);
    if (e == hipSuccess) e = dt.alloc(tb);
    if (e == hipSuccess) e = hipMemcpyAsync(dp.p, perms, (size_t)k * h->n * 4, hipMemcpyHostToDevice, c.st);
    if (e != hipSuccess) return dev_err(e);
    int rc = qap_delta_table_async(h, (const int32_t *)dp.p, k, (int32_t *)dt.p, c.st);
    if (rc != QAP_OK) return rc;
    e = hipMemcpyAsync(table, dt.p, tb, hipMemcpyDeviceToHost, c.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    return dev_err(e);
}

static int host_search(qap_handle h, int algo, int32_t *perms, int32_t k, int32_t iters, int32_t lo,
                       int32_t hi, uint64_t seed, int64_t *costs, int32_t *steps) {
    if (!check_perms(perms, k, h->n)) return QAP_E_NOT_PERM;
    if (k == 0) return QAP_OK;
    HostCall c;
    DevBuf dp, dc, ds;
    const size_t pb = (size_t)k * h->n * 4;
    hipError_t e = c.init();
    if (e == hipSuccess) e = dp.alloc(pb);
    if (e == hipSuccess) e = dc.alloc((size_t)k * 8);
    if (e == hipSuccess) e = ds.alloc((size_t)k * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(dp.p, perms, pb, hipMemcpyHostToDevice, c.st);
    if (e != hipSuccess) return dev_err(e);
    int rc = algo == 0
        ? qap_tabu_async(h, (int32_t *)dp.p, k, iters, lo, hi, seed, 0, (int64_t *)dc.p, (int32_t *)ds.p, c.st)
        : qap_2opt_async(h, (int32_t *)dp.p, k, iters, (int64_t *)dc.p, (int32_t *)ds.p, c.st);
    if (rc != QAP_OK) return rc;
    e = hipMemcpyAsync(perms, dp.p, pb, hipMemcpyDeviceToHost, c.st);
    if (e == hipSuccess) e = hipMemcpyAsync(costs, dc.p, (size_t)k * 8, hipMemcpyDeviceToHost, c.st);
    if (e == hipSuccess && steps) e = hipMemcpyAsync(steps, ds.p, (size_t)k * 4, hipMemcpyDeviceToHost, c.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    return dev_err(e);
}

int qap_2opt(qap_handle h, int32_t *perms, int32_t k, int32_t max_iters, int64_t *costs_out, int32_t *steps_out) {
    if (!h || k < 0 || (k > 0 && (!perms || !costs_out))) return QAP_E_INVALID;
    return host_search(h, 1, perms, k, max_iters, 0, 0, 0, costs_out, steps_out);
}

int qap_tabu(qap_handle h, int32_t *perms, int32_t k, int32_t iters, int32_t lo, int32_t hi, uint64_t seed,
             int64_t *best_costs_out, int32_t *iters_done_out) {
    if (!h || k < 0 || !tenure_args_ok(iters, lo, hi) || (k > 0 && (!perms || !best_costs_out)))
        return QAP_E_INVALID;
    return host_search(h, 0, perms, k, iters, lo, hi, seed, best_costs_out, iters_done_out);
}

}  // extern "C"

// ---- batched tabu over many instances of uneven n

namespace {

// Whether tile shape ri serves this instance in batch_freq_kernel (BATCH_LANES lanes,
// rows 2, 4, 8 or the streamed form).
bool batch_freq_fits(const qap_ctx *h, int ri) {
    if (h->n > WIDE_N) return false;
    // that kernel's own LDS (its marks and reductions, for every shape) comes on top
    const size_t fs = freq_static_lds();
    if (fs >= h->max_smem) return false;
    if (ri == kStream) return h->stream_ok != 0 && stream_smem_bytes(h->n, h->sym) <= h->max_smem - fs;
    if (ri < kBatchFirst || ri > kBatchFirst + 2) return false;
    const TileSet &ts = h->tiles[ri];
    const int rows = kRowsChoices[ri];
    return ts.d_tiles && batch_shape_ok(h->n, rows, ts.ntiles, h->sym) &&
           search_smem_bytes(h->n, rows, BATCH_LANES, h->sym) <= h->max_smem - fs;
}

int batch_create_impl(const qap_handle *hs, int32_t m, const int32_t *k_per, int32_t iters, const int32_t *lo_per,
                      const int32_t *hi_per, const uint64_t *seed_per, const int32_t *rows_per, bool freq,
                      const int32_t *div_per, const int32_t *attr_per, qap_batch_handle *out) {
    if (!hs || !k_per || !lo_per || !hi_per || !seed_per || !out || m < 0 || iters < 0) return QAP_E_INVALID;
    *out = nullptr;
    std::vector<Item> items;
    std::vector<WideTable> wide_tables;
    long long perm_off = 0, out_off = 0, table_off = 0, tile_off = 0, freq_off = 0, uloc_off = 0;
    size_t gsmem[BV_COUNT] = {}, tsmem = 0, fsmem = 0;
    for (int i = 0; i < m; ++i) {
        qap_ctx *h = hs[i];
        if (!h || k_per[i] < 0 || !tenure_args_ok(iters, lo_per[i], hi_per[i])) return QAP_E_INVALID;
        const int div = div_per ? div_per[i] : 0, attr = attr_per ? attr_per[i] : 0;
        if (div < 0 || attr < 0 || attr > 2) return QAP_E_INVALID;
        int ri = rows_per && rows_per[i] != 0 ? rows_index(rows_per[i]) : batch_shape(h);
        if (freq && !(rows_per && rows_per[i] != 0) && ri >= 0 && !batch_freq_fits(h, ri)) {
            // the library's shape needs more than BATCH_LANES lanes: the next larger tile
            // that fits, else the streamed form
            int alt = -1;
            for (int c = ri + 1; c <= kBatchFirst + 2 && alt < 0; ++c)
                if (batch_freq_fits(h, c)) alt = c;
            ri = alt >= 0 ? alt : kStream;
        }
        if (ri < 0 || !(freq ? batch_freq_fits(h, ri) : batch_fits(h, ri))) return QAP_E_UNSUPPORTED;
        const bool streamed = ri == kStream;
        const TileSet &ts = shape_tiles(h, ri);
        const int rows = streamed ? STREAM_ROWS : kRowsChoices[ri];
        const int var = batch_variant(h->n, rows, streamed, ts.ntiles, h->sym);
        const size_t sm = streamed ? stream_smem_bytes(h->n, h->sym)
                                   : search_smem_bytes(h->n, rows, freq ? BATCH_LANES : batch_variant_lanes(var),
                                                       h->sym);
        if (freq)
            fsmem = std::max(fsmem, sm);
        else
            gsmem[var] = std::max(gsmem[var], sm);
        const bool wide = h->n > WIDE_N;
        if (wide) {
            if (k_per[i] > 0)
                wide_tables.push_back(WideTable{h->d_mats, h->n, h->m, k_per[i], h->sym, perm_off, table_off});
        } else {
            tsmem = std::max(tsmem, table_smem_bytes(h->n));
        }
        for (int j = 0; j < k_per[i]; ++j) {
            Item it{};
            it.mats = h->d_mats;
            it.tiles = ts.d_tiles;
            it.n = h->n;
            it.m = h->m;
            it.sym = h->sym;
            it.ntiles = ts.ntiles;
            it.ninterior = ts.ninterior;
            it.rows = streamed ? STREAM_ROWS : kRowsChoices[ri];
            it.stream = streamed ? 1 : 0;
            if (streamed) {
                it.tile_off = tile_off;
                tile_off += stream_tile_int4(ts.ntiles);
            }
            it.iters = iters;
            it.lo = lo_per[i];
            it.hi = hi_per[i];
            it.seed = seed_per[i];
            it.start_id = j;
            it.perm_off = perm_off;
            it.out_off = out_off;
            it.table_off = table_off;
            if (freq) {
                // offsets into the plan's count and unit-location buffers, made absolute
                // once they are allocated
                it.div = div;
                it.attr = attr;
                it.freq_off = freq_off;
                freq_off += h->m;
                if (attr == 2) {
                    it.uloc_off = uloc_off;
                    uloc_off += (long long)h->n * h->n;
                }
            }
            items.push_back(it);
            perm_off += h->n;
            out_off += 1;
            table_off += h->m;
        }
    }
    // grouped by kernel variant; longest first inside a group (the hardware starts blocks
    // in index order)
    std::stable_sort(items.begin(), items.end(), [freq](const Item &a, const Item &b) {
        const int va = freq ? 0 : item_variant(a), vb = freq ? 0 : item_variant(b);
        if (va != vb) return va < vb;
        return (long long)a.n * a.n > (long long)b.n * b.n;
    });
    qap_batch *b = new (std::nothrow) qap_batch;
    if (!b) return QAP_E_NOMEM;
    b->count = (int)items.size();
    b->perm_ints = perm_off;
    b->table_ints = table_off;
    b->tile_int4 = tile_off;
    b->table_smem = tsmem;
    b->freq_mode = freq;
    b->freq_smem = fsmem;
    b->freq_ints = freq_off;
    b->wide_tables = wide_tables;
    for (int i = (int)items.size() - 1; i >= 0; --i) {
        const int v = item_variant(items[i]);
        if (v < 0) continue;   // (not reached: batch_fits and batch_freq_fits turn such shapes away)
        b->group_begin[v] = i;
        ++b->group_count[v];
    }
    int ngroups = 0;
    long long work[BV_COUNT] = {};   // a group's work estimate: the sum of n^2 over its searches
    int order[BV_COUNT];
    for (int v = 0; v < BV_COUNT; ++v) {
        b->group_smem[v] = gsmem[v];
        ngroups += b->group_count[v] > 0;
        for (int i = 0; i < b->group_count[v]; ++i) {
            const long long nn = items[b->group_begin[v] + i].n;
            work[v] += nn * nn;
        }
        order[v] = v;
    }
    std::stable_sort(order, order + BV_COUNT, [&](int x, int y) { return work[x] > work[y]; });
    if (!freq && ngroups > 0) {
        b->nlanes = std::min(ngroups, side_lanes());
        long long load[BV_COUNT] = {};
        int lane_of[BV_COUNT], per_lane[BV_COUNT] = {};
        for (int g = 0; g < ngroups; ++g) {   // largest first, each to the least loaded lane
            int l = 0;
            for (int x = 1; x < b->nlanes; ++x)
                if (load[x] < load[l]) l = x;
            lane_of[order[g]] = l;
            load[l] += work[order[g]];
            ++per_lane[l];
        }
        // Launch order: the lanes by their longest search, longest first, and inside a lane
        // its variants the same way.  A variant of long searches also has the largest
        // blocks (most lanes and LDS), which start only on nearly empty compute units;
        // launched first they take units before the smaller blocks of the other lanes
        // fill them (uneven batch: 138.4 -> 134.4 ms per step).
        auto longest = [&](int v) { return (long long)items[b->group_begin[v]].n; };   // items sorted by n
        long long lane_max[BV_COUNT] = {};
        for (int g = 0; g < ngroups; ++g) {
            const int l = lane_of[order[g]];
            lane_max[l] = std::max(lane_max[l], longest(order[g]));
        }
        int lane_rank[BV_COUNT];
        for (int l = 0; l < b->nlanes; ++l) lane_rank[l] = l;
        std::stable_sort(lane_rank, lane_rank + b->nlanes, [&](int x, int y) { return lane_max[x] > lane_max[y]; });
        int slot_of[BV_COUNT];
        for (int i = 0; i < b->nlanes; ++i) slot_of[lane_rank[i]] = i;
        for (int i = 0; i < b->nlanes; ++i) b->lane_begin[i + 1] = b->lane_begin[i] + per_lane[lane_rank[i]];
        int in_lane[BV_COUNT];
        for (int g = 0; g < ngroups; ++g) in_lane[g] = order[g];
        std::stable_sort(in_lane, in_lane + ngroups, [&](int x, int y) { return longest(x) > longest(y); });
        int fill[BV_COUNT] = {};
        for (int g = 0; g < ngroups; ++g) {
            const int v = in_lane[g], i = slot_of[lane_of[v]];
            b->lane_groups[b->lane_begin[i] + fill[i]++] = v;
        }
    }
    hipError_t e = hipSuccess;
    if (b->nlanes > 1) {
        e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        for (int l = 0; l < b->nlanes && e == hipSuccess; ++l) {
            e = hipStreamCreateWithFlags(&b->side[l], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[l], hipEventDisableTiming);
        }
    }
    if (b->count > 0) {
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_items, items.size() * sizeof(Item));
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_table, (size_t)table_off * sizeof(int32_t) + 16);
        if (e == hipSuccess && tile_off > 0) e = hipMalloc((void **)&b->d_tile_work, (size_t)tile_off * sizeof(int4));
        if (e == hipSuccess && freq) e = hipMalloc((void **)&b->d_freq, (size_t)freq_off * sizeof(int32_t) + 16);
        if (e == hipSuccess && uloc_off > 0)
            e = hipMalloc((void **)&b->d_uloc, (size_t)uloc_off * sizeof(int32_t) + 16);
        if (e == hipSuccess && freq)
            for (Item &it : items) {
                it.freq = b->d_freq + it.freq_off;
                if (it.attr == 2) it.uloc = b->d_uloc + it.uloc_off;
            }
        if (e == hipSuccess) e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        qap_batch_destroy(b);
        return dev_err(e);
    }
    *out = b;
    return QAP_OK;
}

}  // namespace

extern "C" int qap_batch_create(const qap_handle *hs, int32_t m, const int32_t *k_per, int32_t iters,
                                const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                                const int32_t *rows_per, qap_batch_handle *out) {
    return batch_create_impl(hs, m, k_per, iters, lo_per, hi_per, seed_per, rows_per, false, nullptr, nullptr, out);
}

extern "C" int qap_batch_create_freq(const qap_handle *hs, int32_t m, const int32_t *k_per, int32_t iters,
                                     const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                                     const int32_t *rows_per, const int32_t *div_per, const int32_t *attr_per,
                                     qap_batch_handle *out) {
    return batch_create_impl(hs, m, k_per, iters, lo_per, hi_per, seed_per, rows_per, true, div_per, attr_per, out);
}

extern "C" int qap_batch_freq_async(qap_batch_handle b, int32_t *d_freq, void *stream) {
    if (!b || !b->freq_mode || (b->freq_ints > 0 && !d_freq)) return QAP_E_INVALID;
    if (b->freq_ints == 0) return QAP_OK;
    return dev_err(hipMemcpyAsync(d_freq, b->d_freq, (size_t)b->freq_ints * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

extern "C" int qap_batch_size(qap_batch_handle b, int64_t *starts_out, int64_t *perm_ints_out) {
    if (!b) return QAP_E_INVALID;
    if (starts_out) *starts_out = b->count;
    if (perm_ints_out) *perm_ints_out = b->perm_ints;
    return QAP_OK;
}

extern "C" int qap_batch_groups(qap_batch_handle b, int32_t *count_out) {
    if (!b) return QAP_E_INVALID;
    if (b->freq_mode) {   // one launch of every search: the searches per tile shape
        if (count_out) {
            for (int v = 0; v < BV_COUNT; ++v) count_out[v] = 0;
            for (int v = 0; v < BV_COUNT; ++v) {
                if (!b->group_count[v]) continue;
                const int rows = v == BV_R4 || v == BV_R4_256 || v == BV_R4_768 ? 4 : (v == BV_R8 ? 8 : 2);
                count_out[v == BV_STREAM ? BV_STREAM : (rows == 2 ? BV_R2 : (rows == 4 ? BV_R4 : BV_R8))] +=
                    b->group_count[v];
            }
        }
        return b->count > 0 ? 1 : 0;
    }
    int groups = 0;
    for (int v = 0; v < BV_COUNT; ++v) {
        if (count_out) count_out[v] = b->group_count[v];
        groups += b->group_count[v] > 0;
    }
    return groups;
}

extern "C" int qap_batch_tables_async(qap_batch_handle b, const int32_t *d_perms, void *stream) {
    if (!b || (b->count > 0 && !d_perms)) return QAP_E_INVALID;
    if (b->count == 0) return QAP_OK;
    const hipStream_t st = (hipStream_t)stream;
    // the searches above WIDE_N come last (their variant is the last one)
    const int narrow = b->count - (b->freq_mode ? 0 : b->group_count[BV_WIDE]);
    BatchArgs a{b->d_items, narrow, const_cast<int32_t *>(d_perms), nullptr, nullptr, b->d_table, b->d_tile_work};
    hipError_t e = launch_table_batch(a, b->table_smem, st);
    for (size_t i = 0; i < b->wide_tables.size() && e == hipSuccess; ++i) {
        const WideTable &w = b->wide_tables[i];
        const TableArgs ta{w.mats, d_perms + w.perm_off, nullptr, b->d_table + w.table_off, w.n, w.m, w.k, w.sym};
        e = launch_table(ta, st);
    }
    return dev_err(e);
}

extern "C" int qap_batch_search_async(qap_batch_handle b, int32_t *d_perms, int64_t *d_best, int32_t *d_done,
                                      void *stream) {
    if (!b || (b->count > 0 && (!d_perms || !d_best))) return QAP_E_INVALID;
    if (b->count == 0) return QAP_OK;
    hipStream_t st = (hipStream_t)stream;
    if (b->freq_mode) {
        BatchArgs a{b->d_items, b->count, d_perms, d_best, d_done, b->d_table, b->d_tile_work};
        return dev_err(launch_batch_freq(a, b->freq_smem, st));
    }
    const bool fork = b->nlanes > 1;
    hipError_t e = fork ? hipEventRecord(b->ev_fork, st) : hipSuccess;
    for (int l = 0; l < b->nlanes && e == hipSuccess; ++l) {
        hipStream_t ls = fork ? b->side[l] : st;
        if (fork) e = hipStreamWaitEvent(ls, b->ev_fork, 0);
        for (int g = b->lane_begin[l]; g < b->lane_begin[l + 1] && e == hipSuccess; ++g) {
            const int v = b->lane_groups[g];
            BatchArgs a{b->d_items + b->group_begin[v], b->group_count[v], d_perms, d_best, d_done, b->d_table,
                        b->d_tile_work};
            e = launch_batch_group(v, a, b->group_smem[v], ls);
        }
        if (fork && e == hipSuccess) e = hipEventRecord(b->ev_join[l], ls);
    }
    // the joins after every lane's launches, so that no wait of the caller's stream sits
    // in a hardware queue ahead of a lane's kernels
    for (int l = 0; fork && l < b->nlanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(st, b->ev_join[l], 0);
    return dev_err(e);
}

extern "C" int qap_batch_run_async(qap_batch_handle b, int32_t *d_perms, int64_t *d_best, int32_t *d_done,
                                   void *stream) {
    int rc = qap_batch_tables_async(b, d_perms, stream);
    return rc == QAP_OK ? qap_batch_search_async(b, d_perms, d_best, d_done, stream) : rc;
}

extern "C" int qap_batch_destroy(qap_batch_handle b) {
    if (!b) return QAP_OK;
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->d_tile_work) (void)hipFree(b->d_tile_work);
    if (b->d_freq) (void)hipFree(b->d_freq);
    if (b->d_uloc) (void)hipFree(b->d_uloc);
    for (int v = 0; v < BV_COUNT; ++v) {
        if (b->side[v]) (void)hipStreamDestroy(b->side[v]);
        if (b->ev_join[v]) (void)hipEventDestroy(b->ev_join[v]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    delete b;
    return QAP_OK;
}

extern "C" int qap_tabu_batch_concat(const qap_handle *hs, int32_t m, int32_t *perms, const int32_t *k_per,
                                     int32_t iters, const int32_t *lo_per, const int32_t *hi_per,
                                     const uint64_t *seed_per, int64_t *best_out, int32_t *done_out) {
    if (!hs || !k_per || (m > 0 && (!perms || !best_out))) return QAP_E_INVALID;
    long long off = 0;
    for (int i = 0; i < m; ++i) {
        if (!hs[i] || k_per[i] < 0) return QAP_E_INVALID;
        if (!check_perms(perms + off, k_per[i], hs[i]->n)) return QAP_E_NOT_PERM;
        off += (long long)k_per[i] * hs[i]->n;
    }
    qap_batch_handle b = nullptr;
    int rc = qap_batch_create(hs, m, k_per, iters, lo_per, hi_per, seed_per, nullptr, &b);
    if (rc != QAP_OK) return rc;
    HostCall c;
    DevBuf dp, db, dd;
    hipError_t e = c.init();
    if (e == hipSuccess) e = dp.alloc((size_t)b->perm_ints * 4);
    if (e == hipSuccess) e = db.alloc((size_t)b->count * 8);
    if (e == hipSuccess) e = dd.alloc((size_t)b->count * 4);
    if (e == hipSuccess && b->count > 0)
        e = hipMemcpyAsync(dp.p, perms, (size_t)b->perm_ints * 4, hipMemcpyHostToDevice, c.st);
    if (e == hipSuccess) {
        rc = qap_batch_run_async(b, (int32_t *)dp.p, (int64_t *)db.p, (int32_t *)dd.p, c.st);
        if (rc == QAP_OK && b->count > 0) {
            e = hipMemcpyAsync(perms, dp.p, (size_t)b->perm_ints * 4, hipMemcpyDeviceToHost, c.st);
            if (e == hipSuccess) e = hipMemcpyAsync(best_out, db.p, (size_t)b->count * 8, hipMemcpyDeviceToHost, c.st);
            if (e == hipSuccess && done_out)
                e = hipMemcpyAsync(done_out, dd.p, (size_t)b->count * 4, hipMemcpyDeviceToHost, c.st);
            if (e == hipSuccess) e = hipStreamSynchronize(c.st);
        }
    }
    qap_batch_destroy(b);
    if (rc != QAP_OK) return rc;
    return dev_err(e);
}

extern "C" int qap_tabu_batch(const qap_handle *hs, int32_t m, int32_t *const *perms, const int32_t *k_per,
                              int32_t iters, const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                              int64_t *const *best_out) {
    if (!hs || !k_per || m < 0 || (m > 0 && (!perms || !best_out))) return QAP_E_INVALID;
    long long ints = 0, starts = 0;
    for (int i = 0; i < m; ++i) {
        if (!hs[i] || k_per[i] < 0 || (k_per[i] > 0 && (!perms[i] || !best_out[i]))) return QAP_E_INVALID;
        ints += (long long)k_per[i] * hs[i]->n;
        starts += k_per[i];
    }
    // gathered into one concatenated batch, run, and scattered back
    std::vector<int32_t> cat;
    std::vector<int64_t> best;
    try {
        cat.resize((size_t)ints);
        best.resize((size_t)starts);
    } catch (...) {
        return QAP_E_NOMEM;
    }
    long long o = 0;
    for (int i = 0; i < m; ++i) {
        const size_t c = (size_t)k_per[i] * hs[i]->n;
        if (c) std::memcpy(cat.data() + o, perms[i], c * sizeof(int32_t));
        o += (long long)c;
    }
    const int rc = qap_tabu_batch_concat(hs, m, cat.data(), k_per, iters, lo_per, hi_per, seed_per, best.data(),
                                         nullptr);
    if (rc != QAP_OK) return rc;
    long long po = 0, bo = 0;
    for (int i = 0; i < m; ++i) {
        const size_t c = (size_t)k_per[i] * hs[i]->n;
        if (c) std::memcpy(perms[i], cat.data() + po, c * sizeof(int32_t));
        if (k_per[i]) std::memcpy(best_out[i], best.data() + bo, (size_t)k_per[i] * sizeof(int64_t));
        po += (long long)c;
        bo += k_per[i];
    }
    return QAP_OK;
}
