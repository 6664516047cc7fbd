// qap_server.hip -- serving loop for tabu solves of uneven n: continuous batching of
// resumable searches over device-resident state.
//
// Requests are admitted in arrival order while a slot is free and their device
// footprint fits the server's memory pool; a request that does not fit is passed over
// by later ones that do, until it has been passed over kMaxPassOvers times, after which
// nothing behind it is admitted before it (so a large request cannot starve).  Each step
// runs one chunk of every admitted search in a single launch (one workgroup per search,
// each stopping at an iteration boundary once a clock budget is spent) and keeps the
// search's permutation, tabu list and neighbourhood on the device between chunks, so a
// search gives exactly the result it gives when run alone in one go.  Requests that
// arrive while a chunk runs join at the next step; finished searches free their slot and
// memory at once.  Steps are driven either by the caller (qap_server_step) or by the
// server's own host thread (qap_server_start); submissions, polls and cancellations are
// safe from any thread meanwhile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qap.h"
#include "qap_host.h"
#include "qap_internal.h"

using namespace qapk;
using namespace qaph;

namespace {

constexpr size_t kAlign = 256;
// Steps a queued request may be passed over by later ones before admission waits for it.
constexpr int kMaxPassOvers = 8;

size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit sub-allocator over one device allocation; free ranges coalesce on release.
class Arena {
public:
    void init(size_t size) {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
    }
    long long alloc(size_t bytes) {
        bytes = up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, left = it->second - bytes;
            free_.erase(it);
            if (left) free_[off + bytes] = left;
            used_ += bytes;
            return (long long)off;
        }
        return -1;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(bytes);
        used_ -= bytes;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }

private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

// Byte layout of one request's device state inside the pool.  Register-tile searches
// save their neighbourhood as (delta, tabu until) pairs between chunks (st_du); streamed
// searches keep their tiles in tile_work throughout.
struct Layout {
    size_t mats, perm, st_perm, st_bestp, table, st_du, tile_work, freq, uloc, st_mark, total;
};

// own_mats: the request brought its own F and D (a copy lives in the pool); otherwise it
// runs on an existing handle's device matrices.
// freq: the request keeps the frequency memory (counts per packed pair), and with attr 2
// the unit-location table, with attr 1 the unit marks between chunks.
Layout layout_for(int n, bool streamed, int ntiles, bool own_mats = true, bool freq = false, int attr = 0) {
    const size_t m = (size_t)n * (n - 1) / 2;
    Layout L{};
    size_t o = 0;
    L.mats = o;     if (own_mats) o += up((size_t)4 * n * row_stride(n));
    L.perm = o;     o += up((size_t)n * 4);
    L.st_perm = o;  o += up((size_t)n * 4);
    L.st_bestp = o; o += up((size_t)n * 4);
    L.table = o;    o += up(m * 4 + 16);
    L.st_du = o;    if (!streamed) o += up(m * 8 + 16);
    L.tile_work = o; if (streamed) o += up((size_t)stream_tile_int4(ntiles) * sizeof(int4));
    L.freq = o;     if (freq) o += up(m * 4 + 16);
    L.uloc = o;     if (freq && attr == 2) o += up((size_t)n * n * 4);
    L.st_mark = o;  if (freq && attr == 1) o += up((size_t)n * 4);
    L.total = o;
    return L;
}

struct Request {
    int64_t ticket = 0;
    int n = 0, m = 0, sym = 0, rows = 0, iters = 0, lo = 0, hi = 0;
    bool streamed = false;
    uint64_t seed = 0;
    bool freq = false;       // keeps the frequency memory (qap_server_submit_freq)
    int div = 0, attr = 0;
    std::vector<uint8_t> mats;          // own copy of [F | F^T | D | D^T], or empty
    const uint8_t *ext_mats = nullptr;  // else the device matrices of a handle
    std::vector<int32_t> start;
    Layout lay{};
    long long off = -1;
    int slot = -1;
    bool fresh = false;      // admitted, table not built yet
    bool cancelled = false;  // dropped at the next step
    bool inject = false;     // test hook: its device state is corrupted before the next chunk
    int passed_over = 0;     // steps in which a later request was admitted before it
    double t_submit = 0, t_admit = 0;
};

struct Result {
    std::vector<int32_t> perm;
    std::vector<int32_t> freq;   // exchange counts, for requests that kept them
    bool has_freq = false;
    int64_t best = 0;
    int32_t moves = 0;
    int status = QAP_OK;     // QAP_E_DEVICE when the search failed on the device
    double latency_ms = 0, queued_ms = 0;
};

struct Tiles {
    int32_t *d = nullptr;
    int ntiles = 0, ninterior = 0;
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct qap_server {
    int device = 0, max_active = 0;
    size_t max_smem = 0;
    long long budget_ticks = 0;
    hipStream_t st = nullptr;
    uint8_t *pool = nullptr;
    size_t pool_bytes = 0;
    Arena arena;
    // per-slot device arrays: search state, best cost, moves
    SearchState *d_state = nullptr;
    int64_t *d_cost = nullptr;
    int32_t *d_moves = nullptr;
    Item *d_items = nullptr, *d_new = nullptr;
    // pinned host mirrors
    Item *h_items = nullptr, *h_new = nullptr;
    SearchState *h_state = nullptr;
    int64_t *h_cost = nullptr;
    int32_t *h_moves = nullptr;
    std::vector<int> free_slots;
    std::map<int, Tiles> tiles;            // key n * 16 + rows
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::unordered_map<int64_t, Result> done;
    std::unordered_map<int64_t, int> state;   // 0 pending, 1 active, 2 done
    std::unordered_map<int64_t, Request *> live;   // pending and active requests by ticket
    int64_t next_ticket = 1;
    long long chunks = 0, steps = 0, finished = 0, failed = 0, cancelled = 0;
    int max_queued = 1 << 16;
    // mu guards everything above that submit, poll, cancel and step share (queues,
    // result maps, arena, slots, tile lists); step_mu makes steps one at a time
    std::mutex mu, step_mu;
    std::condition_variable cv;
    std::thread driver;
    bool driver_on = false, driver_stop = false;
    int driver_error = QAP_OK;
};

namespace {

const Tiles *tiles_for(qap_server *s, int n, int rows, int *rc) {
    const int key = n * 16 + rows;
    auto it = s->tiles.find(key);
    if (it != s->tiles.end()) return &it->second;
    int ninner = 0;
    std::vector<int32_t> tl = enumerate_tiles(n, rows, &ninner);
    Tiles t;
    t.ntiles = (int)tl.size();
    t.ninterior = ninner;
    hipError_t e = hipMalloc((void **)&t.d, tl.size() * 4 + 16);
    if (e == hipSuccess) e = hipMemcpy(t.d, tl.data(), tl.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (t.d) (void)hipFree(t.d);
        *rc = dev_err(e);
        return nullptr;
    }
    return &s->tiles.emplace(key, t).first->second;
}

// The tile shape a request runs with: the smallest of 2, 4, 8 rows that fits the
// register-tile kernel, else the streamed kernel (rows = -STREAM_ROWS; its wide form
// above WIDE_N); -1 if none.  freq: the request keeps the frequency memory, whose kernel
// holds LDS of its own beside the plan's.
int server_rows(qap_server *s, int n, int sym, int *rc, bool freq = false) {
    *rc = QAP_OK;
    const size_t fs = freq ? freq_static_lds() : 0;
    const size_t room = fs < s->max_smem ? s->max_smem - fs : 0;
    for (int rows : {2, 4, 8}) {
        if (n > WIDE_N) break;
        int ninner = 0;
        const int nt = (int)enumerate_tiles(n, rows, &ninner).size();
        if (batch_shape_ok(n, rows, nt, sym) && search_smem_bytes(n, rows, BATCH_LANES, sym) <= room)
            return tiles_for(s, n, rows, rc) ? rows : -1;
    }
    if (stream_shape_ok(n, sym, room)) return tiles_for(s, n, STREAM_ROWS, rc) ? -STREAM_ROWS : -1;
    *rc = QAP_E_UNSUPPORTED;
    return -1;
}

Item make_item(qap_server *s, const Request *r) {
    const Tiles &ts = s->tiles[r->n * 16 + (r->streamed ? STREAM_ROWS : r->rows)];
    uint8_t *base = s->pool + r->off;
    Item it{};
    it.mats = r->ext_mats ? r->ext_mats : base + r->lay.mats;
    it.tiles = ts.d;
    it.table = reinterpret_cast<const int32_t *>(base + r->lay.table);
    it.perm_in = reinterpret_cast<const int32_t *>(base + r->lay.perm);
    it.perm_out = reinterpret_cast<int32_t *>(base + r->lay.perm);
    it.cost_out = s->d_cost + r->slot;
    it.steps_out = s->d_moves + r->slot;
    it.st = s->d_state + r->slot;
    it.st_perm = reinterpret_cast<int32_t *>(base + r->lay.st_perm);
    it.st_bestp = reinterpret_cast<int32_t *>(base + r->lay.st_bestp);
    it.st_du = reinterpret_cast<int2 *>(base + r->lay.st_du);
    it.stream = r->streamed ? 1 : 0;
    if (r->streamed) {
        it.tile_d = reinterpret_cast<int4 *>(base + r->lay.tile_work);
        it.tile_u = it.tile_d + stream_tile_int4(ts.ntiles) / 2;
    }
    if (r->freq) {
        it.freq = reinterpret_cast<int32_t *>(base + r->lay.freq);
        it.div = r->div;
        it.attr = r->attr;
        if (r->attr == 2) it.uloc = reinterpret_cast<int32_t *>(base + r->lay.uloc);
        if (r->attr == 1) it.st_mark = reinterpret_cast<int32_t *>(base + r->lay.st_mark);
    }
    it.n = r->n;
    it.m = r->m;
    it.sym = r->sym;
    it.ntiles = ts.ntiles;
    it.ninterior = ts.ninterior;
    it.rows = r->streamed ? STREAM_ROWS : r->rows;
    it.iters = r->iters;
    it.lo = r->lo;
    it.hi = r->hi;
    it.seed = r->seed;
    it.start_id = 0;
    it.budget = s->budget_ticks;
    return it;
}

void release(qap_server *s, Request *r) {
    if (r->off >= 0) s->arena.release((size_t)r->off, r->lay.total);
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    r->off = -1;
    r->slot = -1;
}

// Queue a request whose matrices and tile shape are settled (s->mu held by the caller).
int enqueue(qap_server *s, Request *r, int32_t n, const int32_t *start, int32_t iters, int32_t lo, int32_t hi,
            uint64_t seed, int64_t *ticket_out) {
    if ((int64_t)s->pending.size() >= s->max_queued) return QAP_E_BUSY;
    r->n = n;
    r->m = n * (n - 1) / 2;
    r->iters = iters;
    r->lo = lo;
    r->hi = hi;
    r->seed = seed;
    r->start.assign(start, start + n);
    r->ticket = s->next_ticket++;
    r->t_submit = now_ms();
    s->pending.push_back(r);
    s->state[r->ticket] = 0;
    s->live[r->ticket] = r;
    *ticket_out = r->ticket;
    s->cv.notify_all();
    return QAP_OK;
}

// Tile shape and layout of a request (s->mu held); QAP_OK or an error code.
int plan_request(qap_server *s, Request *r, int n) {
    int rc = QAP_OK;
    r->rows = server_rows(s, n, r->sym, &rc, r->freq);
    if (rc != QAP_OK) return rc;
    r->streamed = r->rows < 0;
    const Tiles &ts = s->tiles[n * 16 + (r->streamed ? STREAM_ROWS : r->rows)];
    r->lay = layout_for(n, r->streamed, ts.ntiles, r->ext_mats == nullptr, r->freq, r->attr);
    if (up(r->lay.total) > s->pool_bytes) return QAP_E_NOMEM;   // could never be admitted
    return QAP_OK;
}

// One step: admit, run one chunk of every admitted search, collect the finished ones.
// Called with s->step_mu held; takes s->mu only around the shared state.
int step_locked(qap_server *s, int32_t *active_out, int32_t *pending_out) {
    hipError_t e = hipSuccess;
    int nnew = 0, count = 0, ngroup[3] = {0, 0, 0};
    size_t smem = 0, fsmem = 0, wsmem = 0, tsmem = 0;
    std::vector<Request *> admitted, injected, fresh_wide;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // cancelled searches leave now
        std::vector<Request *> keep;
        for (Request *r : s->active) {
            if (!r->cancelled) { keep.push_back(r); continue; }
            release(s, r);
            delete r;
        }
        s->active.swap(keep);
        // admission in arrival order; a request that does not fit is passed over by later
        // ones that do, until it has waited kMaxPassOvers steps
        std::deque<Request *> still;
        bool blocked = false;
        while (!s->pending.empty()) {
            Request *r = s->pending.front();
            s->pending.pop_front();
            long long off = -1;
            if (!blocked && !s->free_slots.empty()) off = s->arena.alloc(r->lay.total);
            if (off < 0) {
                if (!blocked && ++r->passed_over > kMaxPassOvers) blocked = true;
                still.push_back(r);
                continue;
            }
            r->off = off;
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            r->fresh = true;
            r->t_admit = now_ms();
            s->active.push_back(r);
            s->state[r->ticket] = 1;
            admitted.push_back(r);
        }
        s->pending.swap(still);
        count = (int)s->active.size();
        // one launch per kernel: plain searches up to WIDE_N, then those that keep the
        // frequency memory, then those above WIDE_N (the wide streamed form)
        auto group = [](const Request *r) { return r->n > WIDE_N ? 2 : (r->freq ? 1 : 0); };
        std::stable_sort(s->active.begin(), s->active.end(),
                         [&](const Request *x, const Request *y) { return group(x) < group(y); });
        for (int i = 0; i < count; ++i) {
            Request *r = s->active[i];
            s->h_items[i] = make_item(s, r);
            const int gr = group(r);
            const bool wide = gr == 2;
            ++ngroup[gr];
            size_t &sm = gr == 2 ? wsmem : (gr == 1 ? fsmem : smem);
            sm = std::max(sm, r->streamed ? stream_smem_bytes(r->n, r->sym)
                                          : search_smem_bytes(r->n, r->rows, BATCH_LANES, r->sym));
            if (r->fresh) {
                if (wide) {
                    fresh_wide.push_back(r);
                } else {
                    s->h_new[nnew++] = s->h_items[i];
                    tsmem = std::max(tsmem, table_smem_bytes(r->n));
                }
                r->fresh = false;
            }
            if (r->inject) {
                injected.push_back(r);
                r->inject = false;
            }
        }
    }
    // device work, outside the lock (only this step touches active requests' buffers)
    for (Request *r : admitted) {
        if (e != hipSuccess) break;
        uint8_t *base = s->pool + r->off;
        if (!r->ext_mats)
            e = hipMemcpyAsync(base + r->lay.mats, r->mats.data(), r->mats.size(), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(base + r->lay.perm, r->start.data(), (size_t)r->n * 4, hipMemcpyHostToDevice, s->st);
        SearchState &hs = s->h_state[r->slot];
        hs = SearchState{};
        hs.it = 1;
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_state + r->slot, &hs, sizeof(SearchState), hipMemcpyHostToDevice, s->st);
    }
    if (count > 0 && e == hipSuccess) {
        if (nnew) e = hipMemcpyAsync(s->d_new, s->h_new, (size_t)nnew * sizeof(Item), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_items, s->h_items, (size_t)count * sizeof(Item), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess && nnew) e = launch_table_items(s->d_new, nnew, tsmem, s->st);
        for (Request *r : fresh_wide) {   // Eq. (2) entry by entry above WIDE_N
            if (e != hipSuccess) break;
            uint8_t *base = s->pool + r->off;
            const TableArgs ta{r->ext_mats ? r->ext_mats : base + r->lay.mats,
                               reinterpret_cast<const int32_t *>(base + r->lay.perm), nullptr,
                               reinterpret_cast<int32_t *>(base + r->lay.table), r->n, r->m, 1, r->sym};
            e = launch_table(ta, s->st);
        }
        // test hook: a corrupted saved permutation (every entry 0), which the search
        // detects when it resumes; it then stops with its failure code
        for (Request *r : injected) {
            if (e != hipSuccess) break;
            uint8_t *base = s->pool + r->off;
            e = hipMemsetAsync(base + r->lay.perm, 0, (size_t)r->n * 4, s->st);
            if (e == hipSuccess) e = hipMemsetAsync(base + r->lay.st_perm, 0, (size_t)r->n * 4, s->st);
        }
        if (e == hipSuccess) e = launch_resume(s->d_items, ngroup[0], smem, s->st);
        if (e == hipSuccess) e = launch_resume_freq(s->d_items + ngroup[0], ngroup[1], fsmem, s->st);
        if (e == hipSuccess)
            e = launch_resume_wide(s->d_items + ngroup[0] + ngroup[1], ngroup[2], wsmem, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_state, s->d_state, (size_t)s->max_active * sizeof(SearchState),
                               hipMemcpyDeviceToHost, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_cost, s->d_cost, (size_t)s->max_active * 8, hipMemcpyDeviceToHost, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_moves, s->d_moves, (size_t)s->max_active * 4, hipMemcpyDeviceToHost, s->st);
        if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    }
    if (e != hipSuccess) return dev_err(e);
    // finished searches: their best permutations come back before they are published
    std::vector<Request *> fin;
    std::vector<std::vector<int32_t>> perms;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (count > 0) {
            ++s->steps;
            s->chunks += count;
        }
        for (Request *r : s->active)
            if (s->h_state[r->slot].done) fin.push_back(r);
    }
    perms.resize(fin.size());
    std::vector<std::vector<int32_t>> freqs(fin.size());
    for (size_t i = 0; i < fin.size() && e == hipSuccess; ++i) {
        perms[i].resize(fin[i]->n);
        e = hipMemcpyAsync(perms[i].data(), s->pool + fin[i]->off + fin[i]->lay.perm, (size_t)fin[i]->n * 4,
                           hipMemcpyDeviceToHost, s->st);
        if (e == hipSuccess && fin[i]->freq) {
            freqs[i].resize(fin[i]->m);
            e = hipMemcpyAsync(freqs[i].data(), s->pool + fin[i]->off + fin[i]->lay.freq, (size_t)fin[i]->m * 4,
                               hipMemcpyDeviceToHost, s->st);
        }
    }
    if (e == hipSuccess && !fin.empty()) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return dev_err(e);
    const double t = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<Request *> keep;
    for (Request *r : s->active)
        if (std::find(fin.begin(), fin.end(), r) == fin.end()) keep.push_back(r);
    for (size_t i = 0; i < fin.size(); ++i) {
        Request *r = fin[i];
        s->live.erase(r->ticket);
        if (r->cancelled) {
            s->state.erase(r->ticket);
        } else {
            Result &res = s->done[r->ticket];
            res.perm.swap(perms[i]);
            res.has_freq = r->freq;
            res.freq.swap(freqs[i]);
            res.best = s->h_cost[r->slot];
            res.moves = s->h_moves[r->slot];
            // a search that found its state corrupted stops with moves = -2 (it never
            // starts from an unchecked permutation: submissions are checked on the host)
            res.status = res.moves < 0 ? QAP_E_DEVICE : QAP_OK;
            res.latency_ms = t - r->t_submit;
            res.queued_ms = r->t_admit - r->t_submit;
            s->state[r->ticket] = 2;
            ++(res.status == QAP_OK ? s->finished : s->failed);
        }
        release(s, r);
        delete r;
    }
    s->active.swap(keep);
    if (active_out) *active_out = (int32_t)s->active.size();
    if (pending_out) *pending_out = (int32_t)s->pending.size();
    return (int)fin.size();
}

void driver_loop(qap_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [s] { return s->driver_stop || !s->pending.empty() || !s->active.empty(); });
            if (s->driver_stop) return;
        }
        std::lock_guard<std::mutex> sl(s->step_mu);
        const int rc = step_locked(s, nullptr, nullptr);
        if (rc < 0) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->driver_error = rc;
            return;
        }
    }
}

}  // namespace

extern "C" {

int qap_server_create(int64_t pool_bytes, int32_t max_active, double chunk_ms, qap_server_handle *out) {
    if (!out || pool_bytes <= 0 || max_active <= 0 || chunk_ms < 0) return QAP_E_INVALID;
    *out = nullptr;
    qap_server *s = new (std::nothrow) qap_server;
    if (!s) return QAP_E_NOMEM;
    s->max_active = max_active;
    s->pool_bytes = up((size_t)pool_bytes);
    int smem = 0, khz = 0;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device);
    s->max_smem = (size_t)smem;
    s->budget_ticks = chunk_ms > 0 ? std::max(1LL, (long long)(chunk_ms * khz)) : 0;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&s->pool, s->pool_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_state, (size_t)max_active * sizeof(SearchState));
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_cost, (size_t)max_active * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_moves, (size_t)max_active * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_items, (size_t)max_active * sizeof(Item));
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_new, (size_t)max_active * sizeof(Item));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_items, (size_t)max_active * sizeof(Item));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_new, (size_t)max_active * sizeof(Item));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_state, (size_t)max_active * sizeof(SearchState));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_cost, (size_t)max_active * 8);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_moves, (size_t)max_active * 4);
    if (e != hipSuccess) {
        qap_server_destroy(s);
        return dev_err(e);
    }
    s->arena.init(s->pool_bytes);
    for (int i = max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    *out = s;
    return QAP_OK;
}

int64_t qap_server_footprint(qap_server_handle s, int32_t n, int32_t sym) {
    if (!s || n < 2 || n > QAP_NMAX) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    int rc = QAP_OK;
    const int rows = server_rows(s, n, sym ? 1 : 0, &rc);
    if (rc != QAP_OK) return rc;
    int ninner = 0;
    const int nt = (int)enumerate_tiles(n, rows < 0 ? STREAM_ROWS : rows, &ninner).size();
    return (int64_t)layout_for(n, rows < 0, nt).total;
}

int qap_server_submit_matrices(qap_server_handle s, const int32_t *F, const int32_t *D, int32_t n,
                               const int32_t *start, int32_t iters, int32_t lo, int32_t hi, uint64_t seed,
                               int64_t *ticket_out) {
    if (!s || !F || !D || !start || !ticket_out || n < 2 || n > QAP_NMAX || !tenure_args_ok(iters, lo, hi))
        return QAP_E_INVALID;
    if (!check_perms(start, 1, n)) return QAP_E_NOT_PERM;
    Request *r = new (std::nothrow) Request;
    if (!r) return QAP_E_NOMEM;
    int rc = pack_instance(F, D, n, r->mats, &r->sym);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc == QAP_OK) rc = plan_request(s, r, n);
    if (rc == QAP_OK) rc = enqueue(s, r, n, start, iters, lo, hi, seed, ticket_out);
    if (rc != QAP_OK) delete r;
    return rc;
}

int qap_server_submit(qap_server_handle s, qap_handle h, const int32_t *start, int32_t iters, int32_t lo,
                      int32_t hi, uint64_t seed, int64_t *ticket_out) {
    const uint8_t *mats = nullptr;
    int n = 0, sym = 0, dev = 0;
    if (!s || !start || !ticket_out || !handle_view(h, &mats, &n, &sym, &dev) || !tenure_args_ok(iters, lo, hi))
        return QAP_E_INVALID;
    if (dev != s->device) return QAP_E_INVALID;
    if (!check_perms(start, 1, n)) return QAP_E_NOT_PERM;
    Request *r = new (std::nothrow) Request;
    if (!r) return QAP_E_NOMEM;
    r->ext_mats = mats;
    r->sym = sym;
    std::lock_guard<std::mutex> lk(s->mu);
    int rc = plan_request(s, r, n);
    if (rc == QAP_OK) rc = enqueue(s, r, n, start, iters, lo, hi, seed, ticket_out);
    if (rc != QAP_OK) delete r;
    return rc;
}

int qap_server_submit_freq(qap_server_handle s, qap_handle h, const int32_t *start, int32_t iters, int32_t lo,
                           int32_t hi, uint64_t seed, int32_t div, int32_t attr, int64_t *ticket_out) {
    const uint8_t *mats = nullptr;
    int n = 0, sym = 0, dev = 0;
    if (!s || !start || !ticket_out || !handle_view(h, &mats, &n, &sym, &dev) || !tenure_args_ok(iters, lo, hi) ||
        div < 0 || attr < 0 || attr > 2)
        return QAP_E_INVALID;
    if (dev != s->device) return QAP_E_INVALID;
    if (n > WIDE_N) return QAP_E_UNSUPPORTED;
    if (!check_perms(start, 1, n)) return QAP_E_NOT_PERM;
    Request *r = new (std::nothrow) Request;
    if (!r) return QAP_E_NOMEM;
    r->ext_mats = mats;
    r->sym = sym;
    r->freq = true;
    r->div = div;
    r->attr = attr;
    std::lock_guard<std::mutex> lk(s->mu);
    int rc = plan_request(s, r, n);
    if (rc == QAP_OK) rc = enqueue(s, r, n, start, iters, lo, hi, seed, ticket_out);
    if (rc != QAP_OK) delete r;
    return rc;
}

int qap_server_set_queue_limit(qap_server_handle s, int32_t max_queued) {
    if (!s || max_queued < 1) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->max_queued = max_queued;
    return QAP_OK;
}

int qap_server_step(qap_server_handle s, int32_t *active_out, int32_t *pending_out) {
    if (!s) return QAP_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->driver_on) return QAP_E_INVALID;   // the server's own thread steps it
    }
    std::lock_guard<std::mutex> sl(s->step_mu);
    return step_locked(s, active_out, pending_out);
}

int qap_server_start(qap_server_handle s) {
    if (!s) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->driver_on) return QAP_OK;
    s->driver_stop = false;
    s->driver_error = QAP_OK;
    try {
        s->driver = std::thread(driver_loop, s);
    } catch (...) {
        return QAP_E_NOMEM;
    }
    s->driver_on = true;
    return QAP_OK;
}

int qap_server_stop(qap_server_handle s) {
    if (!s) return QAP_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->driver_on) return QAP_OK;
        s->driver_stop = true;
        s->cv.notify_all();
    }
    s->driver.join();
    std::lock_guard<std::mutex> lk(s->mu);
    s->driver_on = false;
    return s->driver_error;
}

// Shared lookup of qap_server_poll and qap_server_result (s->mu held): 1 and the result
// once finished (the ticket is then forgotten), 0 while queued or running, an error code
// for a search that failed (forgotten too) or an unknown ticket.
static int take_result(qap_server *s, int64_t ticket, Result *out) {
    auto st = s->state.find(ticket);
    if (st == s->state.end()) return QAP_E_INVALID;
    if (st->second != 2) return s->driver_error != QAP_OK ? s->driver_error : 0;
    auto it = s->done.find(ticket);
    *out = std::move(it->second);
    s->done.erase(it);
    s->state.erase(st);
    return out->status == QAP_OK ? 1 : out->status;
}

int qap_server_poll(qap_server_handle s, int64_t ticket, int32_t *best_perm, int64_t *best_cost) {
    if (!s) return QAP_E_INVALID;
    Result r;
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        rc = take_result(s, ticket, &r);
    }
    if (rc == 1) {
        if (best_perm) std::copy(r.perm.begin(), r.perm.end(), best_perm);
        if (best_cost) *best_cost = r.best;
    }
    return rc;
}

int qap_server_poll_freq(qap_server_handle s, int64_t ticket, int32_t *best_perm, int64_t *best_cost,
                         int32_t *freq_out) {
    if (!s) return QAP_E_INVALID;
    Result r;
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // a request that kept no counts is left to qap_server_poll
        auto st = s->state.find(ticket);
        if (freq_out && st != s->state.end() && st->second == 2 && !s->done[ticket].has_freq) return QAP_E_INVALID;
        auto lv = s->live.find(ticket);
        if (freq_out && lv != s->live.end() && !lv->second->freq) return QAP_E_INVALID;
        rc = take_result(s, ticket, &r);
    }
    if (rc == 1) {
        if (best_perm) std::copy(r.perm.begin(), r.perm.end(), best_perm);
        if (best_cost) *best_cost = r.best;
        if (freq_out) std::copy(r.freq.begin(), r.freq.end(), freq_out);
    }
    return rc;
}

int qap_server_result(qap_server_handle s, int64_t ticket, int32_t *perm_out, int64_t *best_out,
                      int32_t *moves_out, double *latency_ms_out) {
    if (!s) return QAP_E_INVALID;
    Result r;
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        rc = take_result(s, ticket, &r);
    }
    if (rc == 1) {
        if (perm_out) std::copy(r.perm.begin(), r.perm.end(), perm_out);
        if (best_out) *best_out = r.best;
        if (moves_out) *moves_out = r.moves;
        if (latency_ms_out) {
            latency_ms_out[0] = r.latency_ms;
            latency_ms_out[1] = r.queued_ms;
        }
    }
    return rc;
}

int qap_server_cancel(qap_server_handle s, int64_t ticket) {
    if (!s) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto st = s->state.find(ticket);
    if (st == s->state.end()) return QAP_E_INVALID;
    if (st->second == 2) return 0;   // finished: the result stays to be collected
    Request *r = s->live[ticket];
    if (st->second == 0) {
        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
        delete r;
    } else {
        r->cancelled = true;   // leaves at the next step boundary
    }
    s->live.erase(ticket);
    s->state.erase(st);
    ++s->cancelled;
    return 1;
}

int qap_server_inject_failure(qap_server_handle s, int64_t ticket) {
    if (!s) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto st = s->state.find(ticket);
    if (st == s->state.end() || st->second != 1) return QAP_E_INVALID;
    s->live[ticket]->inject = true;
    return QAP_OK;
}

int qap_server_stats(qap_server_handle s, int64_t *out) {
    if (!s || !out) return QAP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = (int64_t)s->active.size();
    out[1] = (int64_t)s->pending.size();
    out[2] = (int64_t)s->arena.used();
    out[3] = (int64_t)s->pool_bytes;
    out[4] = s->steps;
    out[5] = s->chunks;
    out[6] = s->finished;
    out[7] = s->failed;
    out[8] = s->cancelled;
    return QAP_OK;
}

int qap_server_destroy(qap_server_handle s) {
    if (!s) return QAP_OK;
    (void)qap_server_stop(s);
    if (s->st) (void)hipStreamSynchronize(s->st);
    for (Request *r : s->pending) delete r;
    for (Request *r : s->active) delete r;
    for (auto &kv : s->tiles)
        if (kv.second.d) (void)hipFree(kv.second.d);
    if (s->pool) (void)hipFree(s->pool);
    if (s->d_state) (void)hipFree(s->d_state);
    if (s->d_cost) (void)hipFree(s->d_cost);
    if (s->d_moves) (void)hipFree(s->d_moves);
    if (s->d_items) (void)hipFree(s->d_items);
    if (s->d_new) (void)hipFree(s->d_new);
    if (s->h_items) (void)hipHostFree(s->h_items);
    if (s->h_new) (void)hipHostFree(s->h_new);
    if (s->h_state) (void)hipHostFree(s->h_state);
    if (s->h_cost) (void)hipHostFree(s->h_cost);
    if (s->h_moves) (void)hipHostFree(s->h_moves);
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return QAP_OK;
}

}  // extern "C"
