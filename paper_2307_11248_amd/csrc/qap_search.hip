// qap_search.hip -- persistent 2opt and tabu search kernels (Secs. 4.1-4.4): one
// workgroup per search, the whole search in one launch, two workgroup barriers per
// iteration.
//
// Data layout
//   * The neighbourhood (one delta per move) lives in registers for the whole search.
//     Lane l owns one tile of the n x n move grid: rows u = ROWS*g .. ROWS*g+ROWS-1 and
//     columns v = 4b .. 4b+3.  Only tiles that hold some u < v exist.  A tile that
//     straddles the diagonal also holds mirror slots (u > v), which carry the same delta
//     and tabu state as (v, u) and so never change the choice, and diagonal slots
//     (u == v), which hold BIG; slots past n (padding) are reset to BIG every iteration.
//   * LDS holds u8 rows of RS = roundup(n, 16) bytes: D and D^T (static) and
//     G = F[p][p], G^T, the flows seen from the locations under the current
//     permutation p (only D and G when F and D are both symmetric).  After a move
//     (r, s), G changes by exchanging rows r, s and columns r, s, done in place.
//   * The tabu state of a move is the iteration at which it becomes free again
//     (Tabuarr of Sec. 4.3), one int32 register beside each delta.
//
// One iteration (p' = p with r and s exchanged, sigma the exchange of r and s):
//   select  each lane folds admissibility and a (delta, key) minimum over its slots; a
//           DPP wave minimum, then the workgroup minimum through LDS        [barrier B1]
//   X       (a) every lane loads the update vectors of its tile's rows and columns
//               A_x = d_xr - d_xs, C_x = d_rx - d_sx, B_x = g_xr - g_xs, E_x = g_rx - g_sx
//               (g = G under p), packed as int16 pairs;
//           (b) the deltas of the moves (u, r) and (u, s) under p', for every u, as four
//               families of n-long u8 dot products (v_dot4) between rows of G, G^T and
//               rows of D, D^T, read under sigma with an O(1) correction; the lanes of
//               one u exchange their dot products by DPP quad permutes and combine them;
//           (c) best-so-far bookkeeping                                       [barrier B2]
//   C       every lane updates its tile: delta += (A_u - A_v)(B_u - B_v)
//           + (C_u - C_v)(E_u - E_v) as two v_pk_sub_i16 and one v_dot2; the rows and
//           columns of r and s are overwritten with the recomputed deltas; the move gets
//           its tabu tenure; G, G^T and p are updated in place.
// The deltas of moves disjoint from {r, s} change only through the k = r, s terms of
// Eq. (2) (Taillard 1991, the elementary tabu search the paper follows); all others are
// recomputed exactly, so every delta stays equal to Eq. (2) of the current permutation.
#include "qap_internal.h"

namespace qapk {

namespace {

typedef short short2_t __attribute__((ext_vector_type(2)));

// Workgroup cap per tile shape, which also caps the registers of a lane: 1024 lanes (4
// waves per SIMD) leave 128 VGPRs, 768 (3 per SIMD) 168, 512 (2) 256.
template <int ROWS>
constexpr int max_lanes() { return ROWS <= 2 ? 1024 : (ROWS == 4 ? 768 : (ROWS <= 8 ? 512 : 256)); }

// (index, family) tasks one lane may carry: enough for 4 n <= 1024 tasks at the lane cap.
template <int ROWS>
constexpr int max_tasks() { return 1024 / max_lanes<ROWS>(); }

template <int CTRL>
__device__ inline int dpp(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

// Minimum of a signed 64-bit key over the wave, by DPP row shifts and row broadcasts;
// every lane returns the minimum.
__device__ inline long long wave_min64(long long v) {
    int lo = (int)v, hi = (int)(v >> 32);
#define QAP_DPP_MIN_STEP(ctrl, rm)                                                        \
    {                                                                                     \
        const int olo = __builtin_amdgcn_update_dpp(lo, lo, ctrl, rm, 0xF, false);      \
        const int ohi = __builtin_amdgcn_update_dpp(hi, hi, ctrl, rm, 0xF, false);      \
        const long long o = ((long long)ohi << 32) | (unsigned)olo;                       \
        const long long c = ((long long)hi << 32) | (unsigned)lo;                         \
        if (o < c) { lo = olo; hi = ohi; }                                                \
    }
    QAP_DPP_MIN_STEP(0x111, 0xF)   // row_shr:1
    QAP_DPP_MIN_STEP(0x112, 0xF)   // row_shr:2
    QAP_DPP_MIN_STEP(0x114, 0xF)   // row_shr:4
    QAP_DPP_MIN_STEP(0x118, 0xF)   // row_shr:8
    QAP_DPP_MIN_STEP(0x142, 0xA)   // row_bcast:15
    QAP_DPP_MIN_STEP(0x143, 0xC)   // row_bcast:31
#undef QAP_DPP_MIN_STEP
    lo = __builtin_amdgcn_readlane(lo, 63);
    hi = __builtin_amdgcn_readlane(hi, 63);
    return ((long long)hi << 32) | (unsigned)lo;
}

// Minimum of a signed 32-bit value over the first `LANES` lanes of the wave (16 or 64),
// by DPP row shifts and row broadcasts; lanes that shift in from outside a row see
// INT32_MAX, the identity of min, so each step is one v_min_i32 with a DPP operand.
template <int LANES>
__device__ inline int wave_min32(int v) {
    constexpr int I = INT32_MAX;
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x118, 0xF, 0xF, false));   // row_shr:8
    if constexpr (LANES == 16) return __builtin_amdgcn_readlane(v, 15);
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// The lowest (delta, key) over the first `LANES` lanes as (delta << 32 | key): the lowest
// delta first, then the lowest key among the lanes that hold it (read from that lane
// when it is alone).  Lanes past LANES are ignored.
template <int LANES>
__device__ inline long long wave_min_pair(int d, int key) {
    const int wd = wave_min32<LANES>(d);
    unsigned long long tie = __ballot(d == wd);
    if constexpr (LANES == 16) tie &= 0xFFFFull;
    int wk;
    if (__builtin_popcountll(tie) == 1)
        wk = __builtin_amdgcn_readlane(key, (int)__builtin_ctzll(tie));
    else
        wk = wave_min32<LANES>(d == wd ? key : KEY_NONE);
    return ((long long)wd << 32) | (unsigned)wk;
}

__device__ inline long long wave_sum64(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Product of two differences of u8 entries (|a|, |b| <= 255): a 24-bit multiply, which
// issues at the full VALU rate (a 32-bit multiply issues at a quarter of it).
__device__ inline int mul8(int a, int b) { return __mul24(a, b); }

__device__ inline int pack16(int lo, int hi) {
    return (int)(((unsigned)hi << 16) | ((unsigned)lo & 0xffffu));
}

__device__ inline int byte_at(unsigned w, int e) { return (int)((w >> (8 * e)) & 0xffu); }

// (x_e - y_e) | (z_e - w_e) << 16 for bytes e of four row words: one packed int16 pair
// of update-vector entries.
__device__ inline int diff_pair(unsigned x, unsigned y, unsigned z, unsigned w, int e) {
    const short2_t a = __builtin_bit_cast(short2_t, pack16(byte_at(x, e), byte_at(z, e)));
    const short2_t b = __builtin_bit_cast(short2_t, pack16(byte_at(y, e), byte_at(w, e)));
    return __builtin_bit_cast(int, a - b);
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
    const unsigned long long span = (unsigned long long)((long long)hi - lo + 1);
    return lo + (int)(((x >> 32) * span) >> 32);
}

__device__ inline unsigned dot_rows(const uint8_t *a, const uint8_t *b, int rs) {
    unsigned acc = 0;
    for (int w = 0; w < rs; w += 16) {
        const uint4 x = *reinterpret_cast<const uint4 *>(a + w);
        const uint4 y = *reinterpret_cast<const uint4 *>(b + w);
        acc = __builtin_amdgcn_udot4(x.x, y.x, acc, false);
        acc = __builtin_amdgcn_udot4(x.y, y.y, acc, false);
        acc = __builtin_amdgcn_udot4(x.z, y.z, acc, false);
        acc = __builtin_amdgcn_udot4(x.w, y.w, acc, false);
    }
    return acc;
}

// Bytes [w, w + 16 * N) of three rows, one uint4 per 16 bytes.
template <int N>
struct RowStep {
    uint4 x[N], y[N], z[N];
};

template <int N>
__device__ inline void load_step(RowStep<N> &q, const uint8_t *a, const uint8_t *b1, const uint8_t *b2, int w) {
#pragma unroll
    for (int h = 0; h < N; ++h) {
        q.x[h] = *reinterpret_cast<const uint4 *>(a + w + 16 * h);
        q.y[h] = *reinterpret_cast<const uint4 *>(b1 + w + 16 * h);
        q.z[h] = *reinterpret_cast<const uint4 *>(b2 + w + 16 * h);
    }
}

template <int N>
__device__ inline void dot_step(const RowStep<N> &q, unsigned &c1, unsigned &c2) {
#pragma unroll
    for (int h = 0; h < N; ++h) {
        c1 = __builtin_amdgcn_udot4(q.x[h].x, q.y[h].x, c1, false);
        c1 = __builtin_amdgcn_udot4(q.x[h].y, q.y[h].y, c1, false);
        c1 = __builtin_amdgcn_udot4(q.x[h].z, q.y[h].z, c1, false);
        c1 = __builtin_amdgcn_udot4(q.x[h].w, q.y[h].w, c1, false);
        c2 = __builtin_amdgcn_udot4(q.x[h].x, q.z[h].x, c2, false);
        c2 = __builtin_amdgcn_udot4(q.x[h].y, q.z[h].y, c2, false);
        c2 = __builtin_amdgcn_udot4(q.x[h].z, q.z[h].z, c2, false);
        c2 = __builtin_amdgcn_udot4(q.x[h].w, q.z[h].w, c2, false);
    }
}

// Two dot products sharing the row `a`, over the first rs bytes (a multiple of 16 N),
// 16 N bytes a step.  Two register sets take turns, so the loads of the next step are in
// flight while the current one is summed, without copying registers between steps.
template <int N>
__device__ inline void dot_rows2_t(const uint8_t *a, const uint8_t *b1, const uint8_t *b2, int rs, unsigned &o1,
                                   unsigned &o2) {
    constexpr int S = 16 * N;
    unsigned c1 = 0, c2 = 0;
    RowStep<N> p, q;
    load_step<N>(p, a, b1, b2, 0);
    for (int w = S;; w += S) {
        if (w < rs) load_step<N>(q, a, b1, b2, w);
        dot_step<N>(p, c1, c2);
        if (w >= rs) break;
        w += S;
        if (w < rs) load_step<N>(p, a, b1, b2, w);
        dot_step<N>(q, c1, c2);
        if (w >= rs) break;
    }
    o1 = c1;
    o2 = c2;
}

// dot_rows2_t for rows of at most MAXB bytes, unrolled over every step: the byte offsets
// are constants, so each load carries its offset in the instruction instead of an address
// add per load; the step count still follows rs (the exits are uniform branches).
template <int N, int MAXB>
__device__ inline void dot_rows2_u(const uint8_t *a, const uint8_t *b1, const uint8_t *b2, int rs, unsigned &o1,
                                   unsigned &o2) {
    constexpr int S = 16 * N;
    static_assert(MAXB % (2 * S) == 0, "whole pairs of steps");
    // an opaque copy of the (uniform) length: the step tests are scalar compares made
    // here, not masks hoisted out of the caller's loop and held in registers throughout
    asm volatile("" : "+s"(rs));
    unsigned c1 = 0, c2 = 0;
    RowStep<N> p, q;
    load_step<N>(p, a, b1, b2, 0);
#pragma unroll
    for (int w = S; w < MAXB; w += 2 * S) {
        if (w < rs) load_step<N>(q, a, b1, b2, w);
        dot_step<N>(p, c1, c2);
        if (w >= rs) break;
        if (w + S < rs) load_step<N>(p, a, b1, b2, w + S);
        dot_step<N>(q, c1, c2);
        if (w + S >= rs) break;
    }
    o1 = c1;
    o2 = c2;
}

// 32 bytes a step (rs a multiple of 32)
__device__ inline void dot_rows2(const uint8_t *a, const uint8_t *b1, const uint8_t *b2, int rs, unsigned &o1,
                                 unsigned &o2) {
    dot_rows2_t<2>(a, b1, b2, rs, o1, o2);
}

// dot_rows2 with one register set carried across steps (the next step's loads go to
// fresh registers that are copied over after the sums): fewer live registers at once,
// at the price of the copies; used by the 2opt kernels, whose tiles leave less room.
__device__ inline void dot_rows2_carry(const uint8_t *a, const uint8_t *b1, const uint8_t *b2, int rs,
                                       unsigned &o1, unsigned &o2) {
    unsigned c1 = 0, c2 = 0;
    RowStep<2> p;
    load_step<2>(p, a, b1, b2, 0);
    for (int w = 32; w <= rs; w += 32) {
        RowStep<2> q = p;
        if (w < rs) load_step<2>(q, a, b1, b2, w);
        dot_step<2>(p, c1, c2);
        p = q;
    }
    o1 = c1;
    o2 = c2;
}

// dot_rows2 for rows of exactly 64 bytes with every load in flight at once: one memory
// latency instead of two (used where the kernel has registers to spare).
__device__ inline void dot_rows2_64(const uint8_t *a, const uint8_t *b1, const uint8_t *b2, unsigned &o1,
                                    unsigned &o2) {
    unsigned c1 = 0, c2 = 0;
    uint4 x[4], y[4], z[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        x[h] = *reinterpret_cast<const uint4 *>(a + 16 * h);
        y[h] = *reinterpret_cast<const uint4 *>(b1 + 16 * h);
        z[h] = *reinterpret_cast<const uint4 *>(b2 + 16 * h);
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        c1 = __builtin_amdgcn_udot4(x[h].x, y[h].x, c1, false);
        c1 = __builtin_amdgcn_udot4(x[h].y, y[h].y, c1, false);
        c1 = __builtin_amdgcn_udot4(x[h].z, y[h].z, c1, false);
        c1 = __builtin_amdgcn_udot4(x[h].w, y[h].w, c1, false);
        c2 = __builtin_amdgcn_udot4(x[h].x, z[h].x, c2, false);
        c2 = __builtin_amdgcn_udot4(x[h].y, z[h].y, c2, false);
        c2 = __builtin_amdgcn_udot4(x[h].z, z[h].z, c2, false);
        c2 = __builtin_amdgcn_udot4(x[h].w, z[h].w, c2, false);
    }
    o1 = c1;
    o2 = c2;
}

// One whole search (or one chunk of it) by the calling workgroup; every lane of the
// block takes part.  MAXT: (index, family) tasks one lane may carry (blockDim.x * MAXT
// >= families * n).  NARROW: the row recomputation reads 16 bytes a step instead of 32
// (for kernels held to 128 VGPRs, where the wider steps spill).  FREQ: tabu keeps the
// frequency memory in a.freq (compiled only into the kernels that need it).
template <int ROWS, bool TABU, int MAXT, bool RESUME, bool STREAM, bool SYM, bool NARROW, bool FREQ = false,
          bool GGLOB = false, bool CTB = false>
__device__ __attribute__((always_inline)) void search_body_t(const Item &a, unsigned char *sm) {
    // CTB: compact tabu state (wide streamed tabu searches without the frequency memory,
    // run whole): a bit per slot in LDS and a ring of recent moves instead of an
    // "until" word per slot streamed with the deltas
    static_assert(!CTB || (TABU && STREAM && GGLOB && !FREQ && !RESUME && ROWS == 8), "compact tabu state");
    __shared__ int s_bad;
    __shared__ int s_chunk_end;   // chunked runs: set by thread 0 once the clock budget is spent
    __shared__ long long s_red2[FREQ ? 16 : 1];   // diversification: wave minima of (count, key)
    __shared__ int s_dd;                          // diversification: delta of the chosen move
    // unit marking: the iteration until which the unit at each location is marked
    __shared__ int s_mark[FREQ ? (GGLOB ? WIDE_MAXN + 8 : 264) : 1];
    const int n = a.n, rs = row_stride(n), L = blockDim.x, t = threadIdx.x;
    const int nb16 = (n + 15) & ~15;   // bytes of a row the dot products read (zero past n)
    const int nb32 = (n + 31) & ~31;   // the same, for the 32-byte steps of the row recomputation
    const int lane = t & 63, wid = t >> 6, W = L >> 6;
    constexpr int sym = SYM ? 1 : 0;   // F and D both symmetric (the caller checked a.sym)
    constexpr int nq = SYM ? 2 : 4, lq = SYM ? 1 : 2;
    // bits of a slot's index inside its tile
    constexpr int KSB = ROWS == 1 ? 2 : (ROWS == 2 ? 3 : (ROWS == 4 ? 4 : 5));
    // Tabu register tiles of up to 4 rows hold each slot as its selection key,
    // delta * 2^KSB + slot (|delta| < 2^26, so keys stay below 2^30 in magnitude): the
    // update scales its (A, C) factors by 2^KSB, and the select needs no shift per slot.
    constexpr bool PS = TABU && !STREAM && ROWS <= 4;
    // the value of a slot that is not a move (diagonal, padding): above every key, and
    // (PS) with room below INT32_MAX for the updates it takes before it is reset
    constexpr int NOMOVE = PS ? (1 << 30) : BIG;
    const int np = padded_n(n, ROWS);
    const Smem S = smem_plan(n, np, L, sym, STREAM, GGLOB);
    SearchState *const st = RESUME ? a.st : nullptr;   // saved state, chunked runs only
    const bool resume = RESUME && st != nullptr && st->it > 1;

    // D and D^T: staged in LDS, or (streamed kernels) read in place from global memory
    const uint8_t *Dm = STREAM ? a.mats + 2 * n * rs : sm + S.d;
    const uint8_t *DmT = STREAM ? a.mats + 3 * n * rs : sm + S.dt;
    // G and G^T in LDS; the wide kernel keeps none: F and F^T in global memory are shared
    // by every search of the instance, and G[x][y] = F[p_x][p_y] is read through the
    // permutation where it is needed
    uint8_t *const gbase = sm;
    const int g_off = S.g, gt_off = S.gt;
    uint8_t *Gm = GGLOB ? nullptr : gbase + g_off, *GmT = GGLOB ? nullptr : gbase + gt_off;
    const uint8_t *FgW = a.mats, *FgWT = a.mats + (size_t)n * rs;
    int *rpr = reinterpret_cast<int *>(sm + S.rpr);
    int *rps = reinterpret_cast<int *>(sm + S.rps);
    int *kc = reinterpret_cast<int *>(sm + S.kc);
    int *acbe = reinterpret_cast<int *>(sm + S.acbe);
    int *perm = reinterpret_cast<int *>(sm + S.perm);
    int *bestp = reinterpret_cast<int *>(sm + S.bestp);
    int *pinv = reinterpret_cast<int *>(sm + S.pinv);
    // (wide kernel) G[x][y] under the current permutation
    auto gF = [&](int x, int y) -> int { return FgW[perm[x] * rs + perm[y]]; };
    int *ten = reinterpret_cast<int *>(sm + S.ten);
    long long *red = reinterpret_cast<long long *>(sm + S.red);
    // compact tabu state: tbits[g * nbw + b] holds the tabu bits of the 8 x 4 slots at
    // tile position (g, b), bit (u % 8) * 4 + v % 4; ring[i % TABU_RING] the move of
    // iteration i; untl[pidx(u, v)] (the tile scratch the until words would take) the
    // iteration until which the latest move of the pair is tabu
    unsigned *tbits = CTB ? reinterpret_cast<unsigned *>(sm + S.tb) : nullptr;
    int *ring = CTB ? reinterpret_cast<int *>(sm + S.ring) : nullptr;
    int *untl = CTB ? reinterpret_cast<int *>(a.tile_u) : nullptr;
    const int nbw = np / TILE_COLS;
    auto tbit_word = [&](int u, int v) -> unsigned * { return tbits + (u >> 3) * nbw + (v >> 2); };
    auto tbit = [&](int u, int v) -> unsigned { return 1u << (((u & 7) << 2) | (v & 3)); };
    // (streamed kernels) the two row dot products of task (u, family q) at
    // xd[q * np + u], made by whole waves
    constexpr bool XW = STREAM;
    int2 *xd = XW ? reinterpret_cast<int2 *>(sm + S.xd) : nullptr;

    // ---- stage D, D^T; read and check the start
    if (!STREAM) {
        const int per = n * rs / 16;
        const uint4 *src = reinterpret_cast<const uint4 *>(a.mats);
        for (int i = t; i < per; i += L) {
            reinterpret_cast<uint4 *>(sm + S.d)[i] = src[2 * per + i];
            if (!sym) reinterpret_cast<uint4 *>(sm + S.dt)[i] = src[3 * per + i];
        }
    }
    if (t == 0) s_bad = 0;
    for (int u = t; u < np; u += L) pinv[u] = -1;
    // (a resumed search keeps its counts and unit-location table from earlier chunks)
    if (FREQ && a.freq && !resume)
        for (int i = t; i < a.m; i += L) a.freq[i] = 0;
    if (FREQ && a.attr == 2 && !resume)
        for (int i = t; i < n * n; i += L) a.uloc[i] = 0;
    __syncthreads();
    const int32_t *pin = resume ? a.st_perm : a.perm_in;
    for (int u = t; u < n; u += L) {
        const int v = pin[u];
        perm[u] = v;
        bestp[u] = resume ? a.st_bestp[u] : v;
        if (v < 0 || v >= n || atomicExch(&pinv[v], u) != -1) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (a.perm_out != a.perm_in)
            for (int u = t; u < n; u += L) a.perm_out[u] = pin[u];
        if (t == 0) {
            *a.cost_out = INT64_MIN;
            if (a.steps_out) *a.steps_out = -2;  // QAP_E_NOT_PERM
            if (st) st->done = 1;
        }
        __syncthreads();
        return;
    }

    // ---- G = F[p][p] and G^T, gathered from the global u8 copies of F and F^T (the wide
    //      kernel keeps no G: it reads F through the permutation where G is needed)
    if constexpr (!GGLOB) {
        const int wpr = rs / 4;  // words per row
        const uint8_t *Fg = a.mats, *FgT = a.mats + (size_t)n * rs;
        for (int i = t; i < n * wpr; i += L) {
            const int row = i / wpr, c0 = (i - row * wpr) * 4;
            const int pr = perm[row];
            unsigned wg = 0, wgt = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = c0 + e;
                if (c < n) {
                    const int pc = perm[c];
                    wg |= (unsigned)Fg[(size_t)pr * rs + pc] << (8 * e);
                    if (!sym) wgt |= (unsigned)FgT[(size_t)pr * rs + pc] << (8 * e);
                }
            }
            reinterpret_cast<unsigned *>(Gm)[i] = wg;
            if (!sym) reinterpret_cast<unsigned *>(GmT)[i] = wgt;
        }
    }
    __syncthreads();

    // ---- RD_u = sum_k D[u][k] G[u][k], CD_u = sum_k D[k][u] G[k][u]; cost (Eq. 1) = sum RD_u
    long long part = 0;
    for (int u = t; u < n; u += L) {
        int rd, cd;
        if constexpr (GGLOB) {
            // G[u][k] = F[p_u][p_k] and G^T[u][k] = F^T[p_u][p_k], byte by byte (once)
            rd = cd = 0;
            const int pu = perm[u];
            for (int k = 0; k < n; ++k) {
                const int pk = perm[k];
                rd += (int)Dm[u * rs + k] * (int)FgW[pu * rs + pk];
                if (!sym) cd += (int)DmT[u * rs + k] * (int)FgWT[pu * rs + pk];
            }
        } else {
            rd = (int)dot_rows(Dm + u * rs, Gm + u * rs, nb16);
            cd = sym ? rd : (int)dot_rows(DmT + u * rs, GmT + u * rs, nb16);
        }
        rpr[u] = rd;
        rps[u] = sym ? rd : cd;
        part += rd;
    }
    part = wave_sum64(part);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    long long cur = 0;
    for (int w = 0; w < W; ++w) cur += red[w];
    long long best = cur;
    if (resume) best = st->best;   // cur is recomputed from the saved permutation
    // per task: RD_u, CD_u, d_uu and g_uu of its u, kept in registers; the streamed kernels
    // below WIDE_N, whose registers are full, keep RD_u and CD_u in LDS (tv: np ints each,
    // written by the lane of family 0 of u) and d_uu there too (tvd, np bytes), and read
    // g_uu from G in LDS
    constexpr bool TVL = STREAM && !GGLOB;
    int *tv = TVL ? reinterpret_cast<int *>(sm + S.tv) : nullptr;
    uint8_t *tvd = TVL ? sm + S.tv + 2 * np * 4 : nullptr;
    int rdv[TVL ? 1 : MAXT], cdv[TVL ? 1 : MAXT], duv[TVL ? 1 : MAXT], guv[TVL ? 1 : MAXT];
    if constexpr (TVL) {
        for (int u = t; u < n; u += L) {
            tv[u] = rpr[u];
            tv[np + u] = rps[u];
            tvd[u] = Dm[u * rs + u];
        }
    } else {
#pragma unroll
        for (int i = 0; i < MAXT; ++i) {
            const int tk = t + i * L;
            rdv[i] = cdv[i] = duv[i] = guv[i] = 0;
            if (tk < nq * n) {
                const int u = tk >> lq;
                rdv[i] = rpr[u];
                cdv[i] = rps[u];
                duv[i] = Dm[u * rs + u];
                guv[i] = GGLOB ? gF(u, u) : Gm[u * rs + u];
            }
        }
    }

    // ---- iteration counter and tenure ring (before the tile loads, so that the Philox
    //      draws do not overlap the loads in flight)
    const long long start_id = a.start_id;
    int it = resume ? st->it : 1, steps = 0;
    const int it_first = it;
    long long clock_end = 0;
    if (RESUME && t == 0) {
        s_chunk_end = 0;
        clock_end = a.budget > 0 ? (long long)wall_clock64() + a.budget : 0;
    }
    int tpos = (it - 1) % L;   // (it - 1) mod L, the tenure ring slot
    if (TABU && tpos != 0) ten[t] = draw_tenure(a.seed, (long long)(it - tpos) + t, start_id, a.lo, a.hi);

    // ---- tiles.  A tile is `ROWS` x 4 neighbourhood slots (u, v) = (u0 + j, v0 + e) held
    //      in registers: dl the deltas, ut the iteration until which the move is tabu.
    //      Register kernels: lane t holds tile t for the whole search.  Streamed kernels:
    //      lane t handles tiles t, t + L, t + 2L, ... one pass at a time, kept in global
    //      memory between passes (tile_d, tile_u, one int4 per (pass, row, lane)).
    constexpr int UTR = TABU ? ROWS : 1;
    constexpr long long NO_MOVE = ((long long)INT32_MAX << 32) | (unsigned)KEY_NONE;
    // slot values of tile (g, b) at the start of the search
    auto load_tile = [&](int (&d)[ROWS][4], int (&u_)[UTR][4], int tu0, int tv0, bool act) {
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = tu0 + j, v = tv0 + e;
                const bool real = act && u < n && v < n && u != v;
                const int ix = real ? (int)pidx(n, u < v ? u : v, u < v ? v : u) : 0;
                if (!STREAM && RESUME && resume) {
                    // (delta, tabu until) of the slot, saved by the previous chunk
                    const int2 du = real ? a.st_du[ix] : make_int2(BIG, INT32_MAX);
                    d[j][e] = !real ? NOMOVE : (PS ? du.x * (1 << KSB) + (j * 4 + e) : du.x);
                    if (TABU) u_[j][e] = du.y;
                } else {
                    d[j][e] = !real ? NOMOVE : (PS ? a.table[ix] * (1 << KSB) + (j * 4 + e) : a.table[ix]);
                    if (TABU) u_[j][e] = real ? 0 : INT32_MAX;
                }
            }
        }
    };
    // lowest admissible slot of a tile at iteration itx (aspiration threshold thr), as
    // (delta << 32 | key), key = u << 9 | v; among equal deltas the lowest slot, i.e. the
    // lowest key.  Up to 8 rows: one 32-bit key per slot, delta * 2^SB + slot, with
    // inadmissible and non-move slots at LIM (above every delta, |delta| < 2^26), so one
    // v_min per slot finds both.  Tabu searches need no clamp of BIG: a slot that is not a
    // move has a tabu state that never expires (INT32_MAX) and BIG is never below the
    // aspiration threshold (best - cur <= 0), so it is never admissible.
    auto tile_min = [&](const int (&d)[ROWS][4], const int (&u_)[UTR][4], int tu0, int tv0, int itx,
                        int thr) -> long long {
        int bd = INT32_MAX, bs = -1;
        if constexpr (PS) {
            // Slot values are keys already (thr scaled the same way).  The admissible slots
            // are the non-tabu ones plus every slot below thr, so their lowest key is the
            // lower of the lowest non-tabu key and, when it is below thr, the lowest key of
            // all: one compare and select per slot, no mask arithmetic.
            int knt[ROWS * 4], kal[ROWS * 4];
#pragma unroll
            for (int j = 0; j < ROWS; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    kal[j * 4 + e] = d[j][e];
                    knt[j * 4 + e] = u_[j][e] <= itx ? d[j][e] : INT32_MAX;
                }
#pragma unroll
            for (int w2 = ROWS * 2; w2 >= 1; w2 >>= 1)
#pragma unroll
                for (int q = 0; q < w2; ++q) {
                    knt[q] = min(knt[q], knt[q + w2]);
                    kal[q] = min(kal[q], kal[q + w2]);
                }
            const int best = kal[0] < thr ? min(knt[0], kal[0]) : knt[0];
            if (best != INT32_MAX) {
                bd = best >> KSB;
                bs = best & ((1 << KSB) - 1);
            }
        } else if constexpr (ROWS <= 8) {
            constexpr int SB = KSB;
            constexpr int LIM = (1 << 26) - 1;
            int best = INT32_MAX;
            if constexpr (ROWS <= 2 && MAXT == 1) {
                // small tiles with registers to spare: a tree of mins (three dependent
                // steps for eight slots instead of a chain of eight)
                int kv[ROWS * 4];
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = d[j][e];
                        const bool adm = TABU ? (u_[j][e] <= itx || x < thr) : true;
                        const int m = adm ? (TABU ? x : min(x, LIM)) : LIM;
                        kv[j * 4 + e] = m * (1 << SB) + (j * 4 + e);
                    }
                }
#pragma unroll
                for (int w2 = ROWS * 2; w2 >= 1; w2 >>= 1)
#pragma unroll
                    for (int q = 0; q < w2; ++q) kv[q] = min(kv[q], kv[q + w2]);
                best = kv[0];
            } else {
#pragma unroll
            for (int j = 0; j < ROWS; ++j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = d[j][e];
                    const bool adm = TABU ? (u_[j][e] <= itx || x < thr) : true;
                    const int m = adm ? (TABU ? x : min(x, LIM)) : LIM;
                    best = min(best, m * (1 << SB) + (j * 4 + e));
                }
            }
            }
            bd = best >> SB;
            bs = best & ((1 << SB) - 1);
            if (bd == LIM) {
                bd = INT32_MAX;
                bs = -1;
            }
        } else {
#pragma unroll
            for (int j = 0; j < ROWS; ++j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = d[j][e];
                    const bool adm = TABU ? (u_[j][e] <= itx || x < thr) : true;
                    if (adm && x < bd) { bd = x; bs = j * 4 + e; }
                }
            }
        }
        const int key = bs < 0 ? KEY_NONE : (((tu0 + (bs >> 2)) << 9) | (tv0 + (bs & 3)));
        return ((long long)bd << 32) | (unsigned)key;
    };
    auto aspiration = [&]() -> int {
        if (!TABU) return 0;
        const long long d = best - cur;  // aspiration: cur + delta < best
        return d < (long long)INT32_MIN ? INT32_MIN : (int)d;
    };
    // the aspiration threshold on key-valued slots: delta < thr exactly when
    // delta * 2^KSB + slot < thr * 2^KSB; below -2^26 no delta reaches it
    auto aspiration_key = [&]() -> int {
        const int th = aspiration();
        return th < -(1 << 26) ? INT32_MIN : th * (1 << KSB);
    };
    // tile_min for the compact tabu state: bit j * 4 + e of tw set = slot (j, e) tabu
    auto tile_min_bits = [&](const int (&d)[ROWS][4], unsigned tw, int tu0, int tv0, int thr) -> long long {
        constexpr int LIM = (1 << 26) - 1;
        int best = INT32_MAX;
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = d[j][e];
                const bool adm = ((tw >> (j * 4 + e)) & 1u) == 0 || x < thr;
                best = min(best, (adm ? x : LIM) * (1 << KSB) + (j * 4 + e));
            }
        int bd = best >> KSB, bs = best & ((1 << KSB) - 1);
        if (bd == LIM) {
            bd = INT32_MAX;
            bs = -1;
        }
        const int key = bs < 0 ? KEY_NONE : (((tu0 + (bs >> 2)) << 9) | (tv0 + (bs & 3)));
        return ((long long)bd << 32) | (unsigned)key;
    };
    const int npass = STREAM ? (a.ntiles + L - 1) / L : 1;
    auto tile_of = [&](int tix, int &g, int &b) {
        const int tv = a.tiles[tix];
        g = tv & 0xffff;
        b = tv >> 16;
    };
    auto tile_addr = [&](int q, int j) { return (q * ROWS + j) * L + t; };

    // register kernels: this lane's tile
    const bool active = !STREAM && t < a.ntiles;
    int g = 0, b = 0;
    if (active) tile_of(t, g, b);
    const int u0 = g * ROWS, v0 = b * TILE_COLS;
    const bool boundary = active && t >= a.ninterior;
    int dl[ROWS][4];
    int ut[UTR][4];
    long long sel = NO_MOVE;   // streamed kernels: this lane's candidate for the next select
    if (!STREAM) {
        load_tile(dl, ut, u0, v0, active);
    } else {
        const int thr = aspiration();
        for (int q = 0; q < npass; ++q) {
            const int tix = t + q * L;
            if (tix >= a.ntiles) break;
            int tg, tb;
            tile_of(tix, tg, tb);
            int d[ROWS][4], u_[UTR][4];
            if (RESUME && resume) {
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    const int4 x = a.tile_d[tile_addr(q, j)];
                    d[j][0] = x.x; d[j][1] = x.y; d[j][2] = x.z; d[j][3] = x.w;
                    if (TABU) {
                        const int4 y = a.tile_u[tile_addr(q, j)];
                        u_[j][0] = y.x; u_[j][1] = y.y; u_[j][2] = y.z; u_[j][3] = y.w;
                    }
                }
            } else {
                load_tile(d, u_, tg * ROWS, tb * TILE_COLS, true);
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    a.tile_d[tile_addr(q, j)] = make_int4(d[j][0], d[j][1], d[j][2], d[j][3]);
                    if (TABU && !CTB) a.tile_u[tile_addr(q, j)] = make_int4(u_[j][0], u_[j][1], u_[j][2], u_[j][3]);
                }
            }
            if constexpr (CTB) {
                // slots that are not moves (diagonal, padding) stay tabu for good
                unsigned w = 0;
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int u = tg * ROWS + j, v = tb * TILE_COLS + e;
                        if (u >= n || v >= n || u == v) w |= 1u << (j * 4 + e);
                    }
                tbits[tg * nbw + tb] = w;
                const long long c = tile_min_bits(d, w, tg * ROWS, tb * TILE_COLS, thr);
                sel = c < sel ? c : sel;
                continue;
            }
            const long long c = tile_min(d, u_, tg * ROWS, tb * TILE_COLS, it, thr);
            sel = c < sel ? c : sel;
        }
    }
    if (t >= W && t < 16) red[t] = NO_MOVE;   // unused wave-minimum slots
    if constexpr (FREQ) {
        if (t >= W && t < 16) s_red2[t] = NO_MOVE;
        for (int u = t; u < np; u += L) s_mark[u] = RESUME && resume && a.st_mark && u < n ? a.st_mark[u] : 0;
    }
    // diversification: the iteration of the last new best (kept between chunks)
    int last_imp = FREQ && RESUME && resume ? st->last_imp : 0;
    bool stopped = false;
    __syncthreads();

    for (;;) {
        if (TABU) {
            if (it > a.iters) break;
        } else {
            if (steps >= (a.iters > 0 ? a.iters : TWO_OPT_MAX_MOVES)) break;
        }
        // chunk end: decided by thread 0 every 16 iterations, read by all after B1
        if (RESUME && t == 0 && clock_end != 0 && it != it_first && (it & 15) == 0)
            s_chunk_end = (long long)wall_clock64() >= clock_end;
        // ---- select: lowest (delta, key) over the admissible slots (streamed kernels
        //      found their lane's candidate while updating the tiles)
        if (!STREAM) sel = active ? tile_min(dl, ut, u0, v0, it, PS ? aspiration_key() : aspiration()) : NO_MOVE;
        const long long kw = wave_min_pair<64>((int)(sel >> 32), (int)(sel & 0xffffffffLL));
        if (lane == 0) red[wid] = kw;
        __syncthreads();  // B1
        if (RESUME && s_chunk_end) break;   // uniform: every lane reads the same word
        // workgroup minimum of the 16 wave-minimum slots (slots past W hold the largest
        // key): lane i of every wave reads slot i, then the same two-pass DPP minimum
        // over the first 16 lanes
        const long long rv = red[lane & 15];
        const long long mk = wave_min_pair<16>((int)(rv >> 32), (int)(rv & 0xffffffffLL));
        // the winner is the same in every lane: keep it in scalar registers
        int dstar = __builtin_amdgcn_readfirstlane((int)(mk >> 32));
        int kstar = __builtin_amdgcn_readfirstlane((int)(mk & 0xffffffffLL));
        bool diversified = false;
        if constexpr (FREQ) {
            if (a.div > 0 && it - last_imp > a.div) {
                // diversification move: the non-tabu pair exchanged least often so far,
                // lowest key on ties (a pair's own slot has a lower key than its mirror
                // slot, so the winner is never a mirror).  The counts are read at device
                // scope: the adds of earlier moves were made in L2.
                long long dsel = NO_MOVE;
                auto consider = [&](int u, int v, int until) {
                    if (u < n && v < n && u != v && until <= it) {
                        const int cnt = __hip_atomic_load(a.freq + pidx(n, min(u, v), max(u, v)),
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const long long c = ((long long)cnt << 32) | (unsigned)((u << 9) | v);
                        dsel = c < dsel ? c : dsel;
                    }
                };
                if constexpr (STREAM) {
                    // the lane's tiles, their tabu state as the last pass stored it
                    for (int q = 0; q < npass; ++q) {
                        const int tix = t + q * L;
                        if (tix >= a.ntiles) break;
                        int tg, tb;
                        tile_of(tix, tg, tb);
                        for (int j = 0; j < ROWS; ++j) {
                            const int4 y = a.tile_u[tile_addr(q, j)];
                            consider(tg * ROWS + j, tb * TILE_COLS, y.x);
                            consider(tg * ROWS + j, tb * TILE_COLS + 1, y.y);
                            consider(tg * ROWS + j, tb * TILE_COLS + 2, y.z);
                            consider(tg * ROWS + j, tb * TILE_COLS + 3, y.w);
                        }
                    }
                } else if (active) {
                    // opaque copies of the tile origin: the count addresses are made here,
                    // not kept through the whole loop as invariants
                    int pu = u0, pv = v0;
                    asm volatile("" : "+v"(pu), "+v"(pv));
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            consider(pu + j, pv + e, ut[j][e]);
                            // one load in flight at a time: this rare path must not add to the
                            // registers the loop holds
                            asm volatile("" ::: "memory");
                        }
                }
                const long long dw = wave_min_pair<64>((int)(dsel >> 32), (int)(dsel & 0xffffffffLL));
                if (lane == 0) s_red2[wid] = dw;
                __syncthreads();  // B1 of the diversification move
                const long long rv2 = s_red2[lane & 15];
                const long long mk2 = wave_min_pair<16>((int)(rv2 >> 32), (int)(rv2 & 0xffffffffLL));
                const int fmin = __builtin_amdgcn_readfirstlane((int)(mk2 >> 32));
                if (fmin != INT32_MAX) {   // else every move is tabu: the ordinary move
                    const int kd = __builtin_amdgcn_readfirstlane((int)(mk2 & 0xffffffffLL));
                    const int ud = kd >> 9, vd = kd & 511;
                    // the lane holding the pair's own slot publishes its delta
                    if constexpr (STREAM) {
                        for (int q = 0; q < npass; ++q) {
                            const int tix = t + q * L;
                            if (tix >= a.ntiles) break;
                            int tg, tb;
                            tile_of(tix, tg, tb);
                            const int j = ud - tg * ROWS, e = vd - tb * TILE_COLS;
                            if (j >= 0 && j < ROWS && e >= 0 && e < TILE_COLS) {
                                const int4 x = a.tile_d[tile_addr(q, j)];
                                s_dd = e == 0 ? x.x : (e == 1 ? x.y : (e == 2 ? x.z : x.w));
                            }
                        }
                    } else if (active && ud >= u0 && ud < u0 + ROWS && vd >= v0 && vd < v0 + TILE_COLS) {
                        int x = 0;
#pragma unroll
                        for (int j = 0; j < ROWS; ++j)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (u0 + j == ud && v0 + e == vd) x = dl[j][e];
                        s_dd = PS ? x >> KSB : x;   // (a key: the delta is its upper bits)
                    }
                    __syncthreads();  // the delta is visible
                    dstar = __builtin_amdgcn_readfirstlane(s_dd);
                    kstar = kd;
                    diversified = true;
                }
            }
        }
        if (TABU ? (dstar == INT32_MAX) : (dstar >= 0)) {
            stopped = true;
            break;
        }
        const int r = min(kstar >> 9, kstar & 511), s = max(kstar >> 9, kstar & 511);
        const bool improved = TABU && (cur + dstar < best);
        cur += dstar;
        if (improved) best = cur;
        if constexpr (FREQ)
            if (improved || diversified) last_imp = it;
        // frequency memory: one more exchange of locations r and s (a vector atomic that
        // nothing waits for; the zeroing above finished before the first barrier)
        if (FREQ && a.freq && t == 0)
            __hip_atomic_fetch_add(a.freq + pidx(n, r, s), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // step record (debugging aid): move it - 1 of the search
        if (FREQ && a.trace && t == 0 && it - 1 < a.trace_cap) {
            long long *tr = a.trace + 4LL * (it - 1);
            tr[0] = r;
            tr[1] = s;
            tr[2] = dstar;
            tr[3] = cur;
        }

        // words of rows r and s of G and G^T for the exchange in C (read now, G is not
        // written before B2); lanes 0 .. 63 of wave 0 (the bytes of n <= 256), all of
        // which hold task 0 (the wide kernel keeps no G, so nothing to exchange)
        const int swl = lane;
        const bool swap_lane = !GGLOB && wid == 0 && lane < rs / 4;
        unsigned sw_r = 0, sw_s = 0, swt_r = 0, swt_s = 0;
        int sw_grr = 0, sw_grs = 0, sw_gsr = 0, sw_gss = 0;
        if (swap_lane) {
            sw_r = reinterpret_cast<const unsigned *>(Gm + r * rs)[swl];
            sw_s = reinterpret_cast<const unsigned *>(Gm + s * rs)[swl];
            swt_r = reinterpret_cast<const unsigned *>(GmT + r * rs)[swl];
            swt_s = reinterpret_cast<const unsigned *>(GmT + s * rs)[swl];
        }
        // The lanes of task u split the bytes they all need and share them by DPP:
        //   q=0: d_ur d_us D_rr D_rs   q=1: d_ru d_su D_sr D_ss
        //   q=2: g_ur g_us G_rr G_rs   q=3: g_ru g_su G_sr G_ss   (g = G under p)
        // (symmetric: q=0 the D bytes, q=1 the G bytes, plus D_ss / G_ss).  Register-tile
        // kernels read them (from LDS) in the task loop below, streamed kernels here.
        auto task_bytes = [&](int u, int q, unsigned (&b)[5]) {
            const bool gfam = !(sym ? q == 0 : q < 2);
            const uint8_t *M = gfam ? Gm : Dm;
            const bool tr = !sym && (q & 1);
            // entry (x, y) of D or G (the wide kernel reads G through F and p)
            auto mat = [&](int x, int y) -> unsigned {
                return GGLOB && gfam ? (unsigned)gF(x, y) : (unsigned)M[x * rs + y];
            };
            b[0] = mat(tr ? r : u, tr ? u : r);
            b[1] = mat(tr ? s : u, tr ? u : s);
            b[2] = mat(tr ? s : r, r);
            b[3] = mat(tr ? s : r, s);
            b[4] = sym ? mat(s, s) : 0;
        };
        // streamed kernels read those bytes of D (the wide kernel also of F) from global
        // memory: all of them before the waves' dot products, each into a register of its
        // own (lanes past the last task read task 0's), so that their latency hides there
        unsigned rbv[XW ? MAXT : 1][5];
        if constexpr (XW) {
#pragma unroll
            for (int i = 0; i < MAXT; ++i) {
                const int tk = t + i * L;
                const bool ok = tk < nq * n;
                task_bytes(ok ? tk >> lq : 0, ok ? tk & (nq - 1) : 0, rbv[i]);
            }
        }
        // ---- X, streamed kernels: the row dot products of every task first, by whole
        //      waves.  Rows of D (and in the wide kernel of G) live in global memory, where
        //      one lane walking a row of its own waits for every step; here a few lanes
        //      share a row (64 bytes each, so a row is read in one contiguous stretch):
        //      eight in the wide kernel, a wave taking eight rows a step (two steps in
        //      flight), family by family with the two side rows held in registers; four
        //      below, with the side rows of D staged in LDS and the rows of the D families
        //      loaded first.  The partial sums are added by DPP and go to LDS for the task
        //      lanes.
        if constexpr (XW && GGLOB) {
            const int oc = lane >> 3, kb = (lane & 7) * 64;
            // wide kernel, no G: with j = p_k, the four families become
            //   f = 0: sum_k G[su][k] D[b][k]     = sum_j F[p_su][j]   D[b][pinv_j]
            //   f = 1: sum_k G^T[su][k] D^T[b][k] = sum_j F^T[p_su][j] D^T[b][pinv_j]
            //   f = 2: sum_k D[u][k] G[b][k]      with G[b][k]   = F[p_b][p_k]
            //   f = 3: sum_k D^T[u][k] G^T[b][k]  with G^T[b][k] = F^T[p_b][p_k]
            // so the rows each task walks are rows of F, F^T, D, D^T (shared by every
            // search of the instance), and only the two side rows of each family are
            // permuted: gathered here into LDS once per iteration (zero past n)
            uint8_t *svb = GGLOB ? sm + S.sv : nullptr;
            if constexpr (GGLOB) {
                const int per = 2 * nb16;
                for (int idx = t; idx < nq * per; idx += L) {
                    const int q = idx / per, rem = idx - q * per, h = rem >= nb16 ? 1 : 0, j = rem - h * nb16;
                    const int f = sym ? 2 * q : q;
                    int v = 0;
                    if (j < n) {
                        const int b = (f < 2) == (h == 0) ? r : s;   // side 1: row r (f < 2) or s
                        v = f == 0   ? Dm[b * rs + pinv[j]]
                            : f == 1 ? DmT[b * rs + pinv[j]]
                            : f == 2 ? FgW[perm[b] * rs + perm[j]]
                                     : FgWT[perm[b] * rs + perm[j]];
                    }
                    svb[(q * 2 + h) * rs + j] = (uint8_t)v;
                }
                __syncthreads();   // the side rows are complete
            }
            for (int q = 0; q < nq; ++q) {
                const int f = sym ? 2 * q : q;
                const uint8_t *Gf = (f & 1) ? GmT : Gm, *Df = (f & 1) ? DmT : Dm;
                const uint8_t *s1 = GGLOB ? svb + (q * 2) * rs : (f < 2 ? Df + r * rs : Gf + s * rs);
                const uint8_t *s2 = GGLOB ? svb + (q * 2 + 1) * rs : (f < 2 ? Df + s * rs : Gf + r * rs);
                uint4 a1[4], a2[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int o = kb + 16 * c;
                    const bool in = o < nb16;   // bytes past nb16 are padding or the next row
                    a1[c] = in ? *reinterpret_cast<const uint4 *>(s1 + o) : make_uint4(0, 0, 0, 0);
                    a2[c] = in ? *reinterpret_cast<const uint4 *>(s2 + o) : make_uint4(0, 0, 0, 0);
                }
                for (int ub = wid * 8; ub < n; ub += 2 * W * 8) {   // uniform per wave
                    unsigned c1[2] = {0, 0}, c2[2] = {0, 0};
                    uint4 x[2][4];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int u = ub + h * W * 8 + oc;
                        const int su = u == r ? s : (u == s ? r : u);
                        const uint8_t *row;
                        if constexpr (GGLOB) {
                            const int psu = u < n ? perm[su] : 0;
                            row = f == 0 ? FgW + psu * rs : (f == 1 ? FgWT + psu * rs : Df + u * rs);
                        } else {
                            row = f < 2 ? Gf + su * rs : Df + u * rs;
                        }
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int o = kb + 16 * c;
                            x[h][c] = u < n && o < nb16 ? *reinterpret_cast<const uint4 *>(row + o)
                                                        : make_uint4(0, 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            c1[h] = __builtin_amdgcn_udot4(x[h][c].x, a1[c].x, c1[h], false);
                            c1[h] = __builtin_amdgcn_udot4(x[h][c].y, a1[c].y, c1[h], false);
                            c1[h] = __builtin_amdgcn_udot4(x[h][c].z, a1[c].z, c1[h], false);
                            c1[h] = __builtin_amdgcn_udot4(x[h][c].w, a1[c].w, c1[h], false);
                            c2[h] = __builtin_amdgcn_udot4(x[h][c].x, a2[c].x, c2[h], false);
                            c2[h] = __builtin_amdgcn_udot4(x[h][c].y, a2[c].y, c2[h], false);
                            c2[h] = __builtin_amdgcn_udot4(x[h][c].z, a2[c].z, c2[h], false);
                            c2[h] = __builtin_amdgcn_udot4(x[h][c].w, a2[c].w, c2[h], false);
                        }
                        // octet sums: quad_perm [1,0,3,2], [2,3,0,1], then the mirrored half row
                        int v1 = (int)c1[h], v2 = (int)c2[h];
                        v1 += dpp<0xB1>(v1); v2 += dpp<0xB1>(v2);
                        v1 += dpp<0x4E>(v1); v2 += dpp<0x4E>(v2);
                        v1 += dpp<0x141>(v1); v2 += dpp<0x141>(v2);
                        const int u = ub + h * W * 8 + oc;
                        if ((lane & 7) == 0 && u < n) xd[q * np + u] = make_int2(v1, v2);
                    }
                }
            }
            __syncthreads();  // the task lanes read xd
        } else if constexpr (XW) {
            // n <= WIDE_N: a row is at most 256 bytes, so four lanes share a row (64 bytes
            // each) and a wave takes 16 rows a step; the two steps of a wave cover every
            // row of a family (2 * 8 waves * 16 rows = 256: streamed kernels run BATCH_LANES
            // lanes).  The side rows r and s of D and D^T (families 0, 1), which every lane
            // needs, are staged in LDS once; the rows of D and D^T that families 2, 3 walk
            // are loaded into registers before that barrier, so a search waits about one
            // memory round trip here.  G and G^T are read from LDS.  Every lane loads from
            // an address inside a row; the bytes past nb16 (a lane's last chunks, for n
            // below 256) are zeroed in the operand read from LDS, and the sums of rows
            // u >= n are not stored.
            // (an opaque copy of the lane's row: the row and LDS addresses are made here each
            // iteration, not kept through the search in registers the kernel does not have)
            int oc = lane >> 2;
            asm volatile("" : "+v"(oc));
            const int kb = (lane & 3) * 64;
            const uint4 z4 = make_uint4(0, 0, 0, 0);
            auto dot16 = [](const uint4 &x, const uint4 &y, unsigned c) {
                c = __builtin_amdgcn_udot4(x.x, y.x, c, false);
                c = __builtin_amdgcn_udot4(x.y, y.y, c, false);
                c = __builtin_amdgcn_udot4(x.z, y.z, c, false);
                return __builtin_amdgcn_udot4(x.w, y.w, c, false);
            };
            // rows u of D or D^T (family q >= nq / 2) for the wave's two steps (rows past n
            // read row 0; chunks past nb16 read the row's first bytes)
            auto load_rows = [&](int q, uint4 (&b)[2][4]) {
                const int f = sym ? 2 * q : q;
                const uint8_t *Df = (f & 1) ? DmT : Dm;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int u = wid * 16 + h * W * 16 + oc;
                    const uint8_t *row = Df + (u < n ? u : 0) * rs;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int o = kb + 16 * c;
                        b[h][c] = *reinterpret_cast<const uint4 *>(row + (o < nb16 ? o : 0));
                    }
                }
            };
            constexpr int nh = nq / 2;   // families with the side rows in D (f < 2)
            uint4 gp[nh][2][4];
#pragma unroll
            for (int q = 0; q < nh; ++q) load_rows(nh + q, gp[q]);
            // side rows [f][r, s] into LDS, 16 bytes a lane
            uint8_t *svd = sm + S.sv;
            const int per = nb16 / 16;
            for (int idx = t; idx < nh * 2 * per; idx += L) {
                const int g = idx / per, c = idx - g * per;
                const uint8_t *Df = (g >> 1) ? DmT : Dm;
                *reinterpret_cast<uint4 *>(svd + g * rs + c * 16) =
                    *reinterpret_cast<const uint4 *>(Df + ((g & 1) ? s : r) * rs + c * 16);
            }
            __syncthreads();   // the side rows are staged
#pragma unroll
            for (int q = 0; q < nq; ++q) {
                const int f = sym ? 2 * q : q;
                const uint8_t *Gf = (f & 1) ? GmT : Gm;
                unsigned c1[2] = {0, 0}, c2[2] = {0, 0};
                if (f < 2) {
                    // rows su of G (or G^T) against the staged side rows r, s of D (or D^T)
                    const uint8_t *sr = svd + (2 * q) * rs, *ss = svd + (2 * q + 1) * rs;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int o = kb + 16 * c, oo = o < nb16 ? o : 0;
                        const uint4 v1 = *reinterpret_cast<const uint4 *>(sr + oo);
                        const uint4 v2 = *reinterpret_cast<const uint4 *>(ss + oo);
                        const uint4 a1 = o < nb16 ? v1 : z4, a2 = o < nb16 ? v2 : z4;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int u = wid * 16 + h * W * 16 + oc;
                            const int su = u >= n ? 0 : (u == r ? s : (u == s ? r : u));
                            const uint4 x = *reinterpret_cast<const uint4 *>(Gf + su * rs + oo);
                            c1[h] = dot16(x, a1, c1[h]);
                            c2[h] = dot16(x, a2, c2[h]);
                        }
                    }
                } else {
                    // rows u of D (or D^T) against the side rows s, r of G (or G^T)
                    uint4 (&b)[2][4] = gp[q - nh];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int o = kb + 16 * c, oo = o < nb16 ? o : 0;
                        const uint4 v1 = *reinterpret_cast<const uint4 *>(Gf + s * rs + oo);
                        const uint4 v2 = *reinterpret_cast<const uint4 *>(Gf + r * rs + oo);
                        const uint4 a1 = o < nb16 ? v1 : z4, a2 = o < nb16 ? v2 : z4;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            c1[h] = dot16(b[h][c], a1, c1[h]);
                            c2[h] = dot16(b[h][c], a2, c2[h]);
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // quad sums: quad_perm [1,0,3,2], then [2,3,0,1]
                    int v1 = (int)c1[h], v2 = (int)c2[h];
                    v1 += dpp<0xB1>(v1); v2 += dpp<0xB1>(v2);
                    v1 += dpp<0x4E>(v1); v2 += dpp<0x4E>(v2);
                    const int u = wid * 16 + h * W * 16 + oc;
                    if ((lane & 3) == 0 && u < n) xd[q * np + u] = make_int2(v1, v2);
                }
            }
            __syncthreads();  // the task lanes read xd
        }
        // ---- X: one (u, family) task per lane: the update vectors of u, and the deltas
        //      of (u, r) and (u, s) under p'
        int colw_addr[MAXT], colw_val[MAXT];
#pragma unroll
        for (int i = 0; i < MAXT; ++i) {
            colw_addr[i] = -1;   // every slot, also those past the last task of this lane
            colw_val[i] = 0;
        }
#pragma unroll
        for (int i = 0; i < MAXT; ++i) {
            int tk = t + i * L;
            // streamed kernels: an opaque copy, so that the LDS addresses made from the task
            // are made here each iteration rather than kept through the search (their
            // registers are full, and spilled addresses cost a memory round trip to reload)
            if constexpr (STREAM) asm volatile("" : "+v"(tk));
            if (tk >= nq * n) break;
            const int u = tk >> lq, q = tk & (nq - 1);
            const int f = sym ? 2 * q : q;   // 0 G.D, 1 G^T.D^T, 2 D.G, 3 D^T.G^T
            const int su = u == r ? s : (u == s ? r : u);
            unsigned rec;
            int ex;
            if constexpr (XW) {
                rec = rbv[i][0] | (rbv[i][1] << 8) | (rbv[i][2] << 16) | (rbv[i][3] << 24);
                ex = (int)rbv[i][4];
            } else {
                const bool gfam = !(sym ? q == 0 : q < 2);
                const uint8_t *M = gfam ? Gm : Dm;
                const bool tr = !sym && (q & 1);
                auto mat = [&](int x, int y) -> unsigned { return (unsigned)M[x * rs + y]; };
                rec = mat(tr ? r : u, tr ? u : r) | (mat(tr ? s : u, tr ? u : s) << 8) |
                      (mat(tr ? s : r, r) << 16) | (mat(tr ? s : r, s) << 24);
                ex = sym ? (int)mat(s, s) : 0;
            }

            // dot products with the O(1) correction sum_k a[sigma k] c[k] = a.c + (a_s - a_r)(c_r - c_s),
            // a a row of G or G^T, c a row of D or D^T:
            //   f = 0: sum_k G'[u][k] D[b][k]    a = G[sigma u],   c = D[b]
            //   f = 1: sum_k G'[k][u] D[k][b]    a = G^T[sigma u], c = D^T[b]
            //   f = 2: sum_k D[u][k] G'[b][k]    a = G[sigma b],   c = D[u]
            //   f = 3: sum_k D[k][u] G'[k][b]    a = G^T[sigma b], c = D^T[u]
            // One loop for every family: the row shared by both sides first, then the side rows.
            // (Issued before the bytes above are used, so their latency hides under the loop.)
            const uint8_t *Gf = (f & 1) ? GmT : Gm, *Df = (f & 1) ? DmT : Dm;
            const uint8_t *shared = f < 2 ? Gf + su * rs : Df + u * rs;
            const uint8_t *side1 = f < 2 ? Df + r * rs : Gf + s * rs;
            const uint8_t *side2 = f < 2 ? Df + s * rs : Gf + r * rs;
            unsigned d1, d2;
            // rows of 64 bytes in one step where the registers allow it (one LDS latency)
            constexpr bool ONE_SHOT = MAXT == 1 && !FREQ && (!NARROW || ROWS <= 2);
            // (rows of n <= WIDE_N bytes: every step unrolled, offsets in the instructions;
            // the kernels with the frequency memory keep the loop, their registers are full)
            if constexpr (XW) {
                const int2 v = xd[q * np + u];   // made by the waves above
                d1 = (unsigned)v.x;
                d2 = (unsigned)v.y;
            } else if (ONE_SHOT && nb32 == 64) {
                dot_rows2_64(shared, side1, side2, d1, d2);
            } else if constexpr (NARROW) {
                dot_rows2_u<1, WIDE_N>(shared, side1, side2, nb16, d1, d2);
            } else if constexpr (!TABU) {
                dot_rows2_carry(shared, side1, side2, nb32, d1, d2);
            } else if constexpr (!FREQ) {
                dot_rows2_u<2, WIDE_N>(shared, side1, side2, nb32, d1, d2);
            } else {
                dot_rows2(shared, side1, side2, nb32, d1, d2);
            }

            unsigned rd_, rdt_, rg_, rgt_, exd = 0, exg = 0;
            if (sym) {
                rd_ = rdt_ = (unsigned)dpp<0xA0>((int)rec);
                rg_ = rgt_ = (unsigned)dpp<0xF5>((int)rec);
                exd = (unsigned)dpp<0xA0>(ex);
                exg = (unsigned)dpp<0xF5>(ex);
            } else {
                rd_ = (unsigned)dpp<0x00>((int)rec);
                rdt_ = (unsigned)dpp<0x55>((int)rec);
                rg_ = (unsigned)dpp<0xAA>((int)rec);
                rgt_ = (unsigned)dpp<0xFF>((int)rec);
            }
            const int d_ur = byte_at(rd_, 0), d_us = byte_at(rd_, 1), D_rr = byte_at(rd_, 2), D_rs = byte_at(rd_, 3);
            const int g_ur = byte_at(rg_, 0), g_us = byte_at(rg_, 1), G_rr = byte_at(rg_, 2), G_rs = byte_at(rg_, 3);
            const int d_ru = byte_at(rdt_, 0), d_su = byte_at(rdt_, 1);
            const int g_ru = byte_at(rgt_, 0), g_su = byte_at(rgt_, 1);
            const int D_sr = sym ? D_rs : byte_at(rdt_, 2), D_ss = sym ? (int)exd : byte_at(rdt_, 3);
            const int G_sr = sym ? G_rs : byte_at(rgt_, 2), G_ss = sym ? (int)exg : byte_at(rgt_, 3);
            if (i == 0) {
                sw_grr = G_rr;
                sw_grs = G_rs;
                sw_gsr = G_sr;
                sw_gss = G_ss;
            }

            // (a_s - a_r) and (c_r - c_s) for the sides r and s, chosen without branches
            const int a0 = (u == r ? G_ss : (u == s ? G_rs : g_us)) - (u == r ? G_sr : (u == s ? G_rr : g_ur));
            const int a1 = (u == r ? G_ss : (u == s ? G_sr : g_su)) - (u == r ? G_rs : (u == s ? G_rr : g_ru));
            const int ar1 = f == 0 ? a0 : (f == 1 ? a1 : (f == 2 ? G_ss - G_sr : G_ss - G_rs));
            const int ar2 = f == 0 ? a0 : (f == 1 ? a1 : (f == 2 ? G_rs - G_rr : G_sr - G_rr));
            const int cr1 = f == 0 ? D_rr - D_rs : (f == 1 ? D_rr - D_sr : (f == 2 ? d_ur - d_us : d_ru - d_su));
            const int cr2 = f == 0 ? D_sr - D_ss : (f == 1 ? D_rs - D_ss : (f == 2 ? d_ur - d_us : d_ru - d_su));
            const int x = (int)d1 + mul8(ar1, cr1);
            const int y = (int)d2 + mul8(ar2, cr2);
            // the four families of u (two when symmetric), shared inside the quad
            int xf[4], yf[4];
            if (sym) {
                xf[0] = xf[1] = dpp<0xA0>(x);   // quad_perm [0,0,2,2]
                yf[0] = yf[1] = dpp<0xA0>(y);
                xf[2] = xf[3] = dpp<0xF5>(x);   // quad_perm [1,1,3,3]
                yf[2] = yf[3] = dpp<0xF5>(y);
            } else {
                xf[0] = dpp<0x00>(x); yf[0] = dpp<0x00>(y);
                xf[1] = dpp<0x55>(x); yf[1] = dpp<0x55>(y);
                xf[2] = dpp<0xAA>(x); yf[2] = dpp<0xAA>(y);
                xf[3] = dpp<0xFF>(x); yf[3] = dpp<0xFF>(y);
            }
            const int A = d_ur - d_us, B = g_ur - g_us, C = d_ru - d_su, E = g_ru - g_su;
            // RD'_u, CD'_u under p'
            int rdn, cdn;
            if (u == r) {
                rdn = xf[2];
                cdn = xf[3];
            } else if (u == s) {
                rdn = yf[2];
                cdn = yf[3];
            } else if constexpr (TVL) {
                rdn = tv[u] - mul8(A, B);
                cdn = tv[np + u] - mul8(C, E);
            } else {
                rdn = rdv[i] - mul8(A, B);
                cdn = cdv[i] - mul8(C, E);
            }
            if constexpr (TVL) {
                // after every lane of u has read them (the lanes of u are one quad of a
                // wave, whose LDS reads and writes take effect in program order)
                if (q == 0) {
                    tv[u] = rdn;
                    tv[np + u] = cdn;
                }
            } else {
                rdv[i] = rdn;
                cdv[i] = cdn;
            }
            // (key-valued tiles: A and C scaled by 2^KSB, |A|, |C| <= 255, so every
            // difference of two still fits 16 bits)
            if (q == 0)
                reinterpret_cast<int2 *>(acbe)[u] =
                    make_int2(PS ? pack16(A * (1 << KSB), C * (1 << KSB)) : pack16(A, C), pack16(B, E));
            if (u == r || u == s) {
                // K_b = RD'_b + CD'_b; every recomputed entry is stored as delta' + K_b, so
                // the tiles subtract K_b alone: here delta'(b, b) = BIG (a diagonal slot;
                // 2^26 for key-valued tiles, whose key 2^30 + slot stays in range)
                // and delta'(r, s) = -dstar (the move undone)
                const int kb = rdn + cdn;
                int *rb = u == r ? rpr : rps;
                if (q == 0) {
                    kc[u == r ? 0 : 1] = kb;
                    rb[u] = (PS ? (1 << 26) : BIG) + kb;
                } else if (q == 1) {
                    rb[u == r ? s : r] = kb - dstar;
                }
            }
            if (q < 2 && u != r && u != s) {
                // delta'(u, b) + RD'_b + CD'_b for b = r (q == 0) or b = s (q == 1)
                const int X = q == 0 ? xf[0] : yf[0], Y = q == 0 ? xf[1] : yf[1];
                const int Z = q == 0 ? xf[2] : yf[2], Wv = q == 0 ? xf[3] : yf[3];
                const int duu = TVL ? (int)tvd[u] : duv[i], guu = TVL ? (int)Gm[u * rs + u] : guv[i];
                const int dbb = q == 0 ? D_rr : D_ss, gbb = q == 0 ? G_ss : G_rr;
                const int dub = q == 0 ? d_ur : d_us, dbu = q == 0 ? d_ru : d_su;
                const int gub = q == 0 ? g_us : g_ur, gbu = q == 0 ? g_su : g_ru;
                const int rowex = mul8(dbu - duu, guu - gbu) + mul8(dbb - dub, gub - gbb);
                const int colex = mul8(dub - duu, guu - gub) + mul8(dbb - dbu, gbu - gbb);
                const int diag = mul8(dbb - duu, guu - gbb) + mul8(dbu - dub, gub - gbu);
                (q == 0 ? rpr : rps)[u] = X + Y + Z + Wv - rdn - cdn - rowex - colex + diag;
            }
            if constexpr (!TVL) {
                if (u == r) guv[i] = G_ss;
                if (u == s) guv[i] = G_rr;
            }
            // this lane's share of exchanging columns r and s of G (and G^T) in row u
            if (!GGLOB && u != r && u != s) {
                if (sym) {
                    colw_addr[i] = g_off + u * rs + (q == 0 ? r : s);
                    colw_val[i] = q == 0 ? g_us : g_ur;
                } else {
                    colw_addr[i] = ((q & 2) ? gt_off : g_off) + u * rs + ((q & 1) ? s : r);
                    colw_val[i] = q == 0 ? g_us : (q == 1 ? g_ur : (q == 2 ? g_su : g_ru));
                }
            }
        }

        // ---- best-so-far and tenures
        if (improved)
            for (int u = t; u < n; u += L) bestp[u] = perm[u == r ? s : (u == s ? r : u)];
        if (TABU && tpos == 0) ten[t] = draw_tenure(a.seed, (long long)it + t, start_id, a.lo, a.hi);
        // unit marking: the two units moved are marked until it + t; they now sit at s
        // and r (thread 0 drew ten[0] itself when tpos is 0; read after B2)
        if constexpr (FREQ)
            if (a.attr == 1 && t == 0) {
                const int tt = it + ten[tpos];
                s_mark[r] = tt;
                s_mark[s] = tt;
            }
        // unit-location pairs: the unit at r may not return to r, nor the one at s to s,
        // until it + t (device-scope stores, complete at B2; read after it at device scope)
        int pr_old = 0, ps_old = 0;   // the units at r and s before the move
        if constexpr (FREQ)
            if (a.attr == 2) {
                pr_old = __builtin_amdgcn_readfirstlane(perm[r]);
                ps_old = __builtin_amdgcn_readfirstlane(perm[s]);
                if (t == 0) {
                    const int tt = it + ten[tpos];
                    __hip_atomic_store(a.uloc + (size_t)pr_old * n + r, tt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(a.uloc + (size_t)ps_old * n + s, tt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        // compact tabu state, for the select of iteration it + 1 (made after B2): the moves
        // of iterations i that expire now (i + t_i == it + 1, so i = it + 1 - t_i with t_i
        // in [lo, hi]) leave the tabu list unless their pair has been made tabu again
        // since (its latest until, a device-scope word, decides); then this move enters it
        // (thread 0 drew ten[0] itself when tpos is 0).  A pair's slot and its mirror
        // change together.
        if constexpr (CTB) {
            const int nxt = it + 1;
            for (int q = t; q <= a.hi - a.lo; q += L) {
                const int i = nxt - a.lo - q;
                if (i < 1 || i >= it) continue;
                const int e = ring[i & (TABU_RING - 1)];
                if (i + (e >> 18) != nxt) continue;
                const int u = (e >> 9) & 511, v = e & 511;
                if ((u == r && v == s) ||
                    __hip_atomic_load(untl + pidx(n, u, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != nxt)
                    continue;
                atomicAnd(tbit_word(u, v), ~tbit(u, v));
                atomicAnd(tbit_word(v, u), ~tbit(v, u));
            }
            if (t == 0) {
                const int tc = ten[tpos];
                ring[it & (TABU_RING - 1)] = (tc << 18) | (r << 9) | s;
                __hip_atomic_store(untl + pidx(n, r, s), it + tc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (tc >= 2) {   // tabu at it + 1
                    atomicOr(tbit_word(r, s), tbit(r, s));
                    atomicOr(tbit_word(s, r), tbit(s, r));
                } else {         // admissible again at it + 1, whatever an earlier move left
                    atomicAnd(tbit_word(r, s), ~tbit(r, s));
                    atomicAnd(tbit_word(s, r), ~tbit(s, r));
                }
            }
        }
        __syncthreads();  // B2

        // ---- C: G, G^T and p follow the move
        if (swap_lane) {
            // rows r and s exchange, with their entries at columns r and s exchanged
            const int wr = swl;
            unsigned nr = sw_s, ns = sw_r, nrt = swt_s, nst = swt_r;
            if ((r >> 2) == wr) {
                const int sh = 8 * (r & 3);
                const unsigned m = ~(0xffu << sh);
                nr = (nr & m) | ((unsigned)sw_gss << sh);
                ns = (ns & m) | ((unsigned)sw_grs << sh);
                nrt = (nrt & m) | ((unsigned)sw_gss << sh);
                nst = (nst & m) | ((unsigned)sw_gsr << sh);
            }
            if ((s >> 2) == wr) {
                const int sh = 8 * (s & 3);
                const unsigned m = ~(0xffu << sh);
                nr = (nr & m) | ((unsigned)sw_gsr << sh);
                ns = (ns & m) | ((unsigned)sw_grr << sh);
                nrt = (nrt & m) | ((unsigned)sw_grs << sh);
                nst = (nst & m) | ((unsigned)sw_grr << sh);
            }
            reinterpret_cast<unsigned *>(Gm + r * rs)[wr] = nr;
            reinterpret_cast<unsigned *>(Gm + s * rs)[wr] = ns;
            if (!sym) {
                reinterpret_cast<unsigned *>(GmT + r * rs)[wr] = nrt;
                reinterpret_cast<unsigned *>(GmT + s * rs)[wr] = nst;
            }
        }
#pragma unroll
        for (int i = 0; i < MAXT; ++i)
            if (colw_addr[i] >= 0) gbase[colw_addr[i]] = (uint8_t)colw_val[i];
        if (t == 0) {
            const int pr = perm[r], ps = perm[s];
            perm[r] = ps;
            perm[s] = pr;
            if (GGLOB) {   // the wide kernel's gathers read p^-1 too
                pinv[ps] = r;
                pinv[pr] = s;
            }
        }
        // ---- C: the tiles follow the move
        const int2 kk = *reinterpret_cast<const int2 *>(kc);
        const int kr = __builtin_amdgcn_readfirstlane(kk.x), ks = __builtin_amdgcn_readfirstlane(kk.y);
        const int until = TABU ? it + ten[tpos] : 0;
        // returns whether the move or its mirror lies in this tile (its tabu state changed)
        auto move_tile = [&](int (&dl)[ROWS][4], int (&ut)[UTR][4], int g, int b, bool boundary) -> bool {
            const int u0 = g * ROWS, v0 = b * TILE_COLS;
            int acu[ROWS], beu[ROWS], acv[4], bev[4];
            {
                const int4 c01 = reinterpret_cast<const int4 *>(acbe + 2 * v0)[0];
                const int4 c23 = reinterpret_cast<const int4 *>(acbe + 2 * v0)[1];
                acv[0] = c01.x; bev[0] = c01.y; acv[1] = c01.z; bev[1] = c01.w;
                acv[2] = c23.x; bev[2] = c23.y; acv[3] = c23.z; bev[3] = c23.w;
                if constexpr (ROWS == 1) {
                    const int2 w = reinterpret_cast<const int2 *>(acbe + 2 * u0)[0];
                    acu[0] = w.x; beu[0] = w.y;
                } else {
#pragma unroll
                    for (int j = 0; j < ROWS; j += 2) {
                        const int4 w = reinterpret_cast<const int4 *>(acbe + 2 * (u0 + j))[0];
                        acu[j] = w.x; beu[j] = w.y; acu[j + 1] = w.z; beu[j + 1] = w.w;
                    }
                }
            }
            // recomputed deltas of rows/columns r and s at this tile's indices (stored + K)
            const int4 rv = *reinterpret_cast<const int4 *>(rpr + v0);
            const int4 sv = *reinterpret_cast<const int4 *>(rps + v0);
            int rpru[ROWS], rpsu[ROWS];
            if constexpr (ROWS == 1) {
                rpru[0] = rpr[u0];
                rpsu[0] = rps[u0];
            } else {
#pragma unroll
                for (int j = 0; j < ROWS; j += 2) {
                    const int2 x2 = *reinterpret_cast<const int2 *>(rpr + u0 + j);
                    const int2 y2 = *reinterpret_cast<const int2 *>(rps + u0 + j);
                    rpru[j] = x2.x; rpru[j + 1] = x2.y;
                    rpsu[j] = y2.x; rpsu[j + 1] = y2.y;
                }
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
            // the rows and columns of r and s; the row/column inside the tile is the same for
            // every lane that holds it, so the slot is picked by a uniform index: tiles of 1
            // and 2 rows select every slot against it (a select per slot, the condition
            // uniform), tiles of 4 and 8 rows are viewed as one vector whose picked slots
            // are written by register-indexed moves, tiles of 16 rows take a scalar branch
            // per row
            const int jr = r % ROWS, js = s % ROWS, er = r & 3, es = s & 3;
            // the value a recomputed delta takes in slot (j, e) (key-valued tiles: its key)
            auto slot_val = [&](int v, int j, int e) { return PS ? v * (1 << KSB) + (j * 4 + e) : v; };
            if constexpr (ROWS <= 2) {
                if (g == r / ROWS) {
                    const int vr[4] = {slot_val(rv.x - kr, jr, 0), slot_val(rv.y - kr, jr, 1),
                                       slot_val(rv.z - kr, jr, 2), slot_val(rv.w - kr, jr, 3)};
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = j == jr ? vr[e] : dl[j][e];
                }
                if (g == s / ROWS) {
                    const int vs[4] = {slot_val(sv.x - ks, js, 0), slot_val(sv.y - ks, js, 1),
                                       slot_val(sv.z - ks, js, 2), slot_val(sv.w - ks, js, 3)};
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = j == js ? vs[e] : dl[j][e];
                }
                if (b == (r >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = e == er ? slot_val(rpru[j] - kr, j, er) : dl[j][e];
                }
                if (b == (s >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = e == es ? slot_val(rpsu[j] - ks, j, es) : dl[j][e];
                }
            } else if constexpr (ROWS <= 8) {
                typedef int tilevec __attribute__((ext_vector_type(ROWS * 4)));
                tilevec tv;
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) tv[j * 4 + e] = dl[j][e];
                if (g == r / ROWS) {
                    tv[jr * 4 + 0] = slot_val(rv.x - kr, jr, 0);
                    tv[jr * 4 + 1] = slot_val(rv.y - kr, jr, 1);
                    tv[jr * 4 + 2] = slot_val(rv.z - kr, jr, 2);
                    tv[jr * 4 + 3] = slot_val(rv.w - kr, jr, 3);
                }
                if (g == s / ROWS) {
                    tv[js * 4 + 0] = slot_val(sv.x - ks, js, 0);
                    tv[js * 4 + 1] = slot_val(sv.y - ks, js, 1);
                    tv[js * 4 + 2] = slot_val(sv.z - ks, js, 2);
                    tv[js * 4 + 3] = slot_val(sv.w - ks, js, 3);
                }
                if (b == (r >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j) tv[j * 4 + er] = slot_val(rpru[j] - kr, j, er);
                }
                if (b == (s >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j) tv[j * 4 + es] = slot_val(rpsu[j] - ks, j, es);
                }
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) dl[j][e] = tv[j * 4 + e];
            } else {
            if (g == r / ROWS) {
                const int vr[4] = {rv.x - kr, rv.y - kr, rv.z - kr, rv.w - kr};
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
                    if (j == jr) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = vr[e];
                    }
            }
            if (g == s / ROWS) {
                const int vs[4] = {sv.x - ks, sv.y - ks, sv.z - ks, sv.w - ks};
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
                    if (j == js) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dl[j][e] = vs[e];
                    }
            }
            if (b == (r >> 2)) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e == er) {
#pragma unroll
                        for (int j = 0; j < ROWS; ++j) dl[j][e] = rpru[j] - kr;
                    }
            }
            if (b == (s >> 2)) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e == es) {
#pragma unroll
                        for (int j = 0; j < ROWS; ++j) dl[j][e] = rpsu[j] - ks;
                    }
            }
            }
            bool tabu_set = false;
            if (FREQ && TABU && a.attr == 1) {
                // unit marking: a slot is tabu while either of its units is marked; only the
                // slots in the rows and columns of r and s changed units or marks
                if (g == r / ROWS || g == s / ROWS || b == (r >> 2) || b == (s >> 2)) {
                    int mu[ROWS], mv[4];
#pragma unroll
                    for (int j = 0; j < ROWS; ++j) mu[j] = s_mark[u0 + j];
#pragma unroll
                    for (int e = 0; e < 4; ++e) mv[e] = s_mark[v0 + e];
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int u = u0 + j, v = v0 + e;
                            if ((u == r || u == s || v == r || v == s) && u < n && v < n && u != v)
                                ut[j][e] = max(mu[j], mv[e]);
                        }
                    tabu_set = true;
                }
            } else if (FREQ && TABU && a.attr == 2) {
                // unit-location pairs: a slot is tabu when both of its units would return to
                // a location they left; only the slots in the rows and columns of r and s
                // changed units or table entries.  The units at other rows and columns are
                // read from p (only p[r] and p[s] change in this phase).
                if (g == r / ROWS || g == s / ROWS || b == (r >> 2) || b == (s >> 2)) {
                    int pu[ROWS], pv[4];
#pragma unroll
                    for (int j = 0; j < ROWS; ++j) {
                        const int x = u0 + j;
                        pu[j] = x == r ? ps_old : (x == s ? pr_old : (x < n ? perm[x] : 0));
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = v0 + e;
                        pv[e] = x == r ? ps_old : (x == s ? pr_old : (x < n ? perm[x] : 0));
                    }
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int u = u0 + j, v = v0 + e;
                            if ((u == r || u == s || v == r || v == s) && u < n && v < n && u != v) {
                                const int xa = __hip_atomic_load(a.uloc + (size_t)pu[j] * n + v, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                                const int xb = __hip_atomic_load(a.uloc + (size_t)pv[e] * n + u, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                                ut[j][e] = min(xa, xb);
                            }
                        }
                    tabu_set = true;
                }
            } else if (TABU && !CTB) {
                // the move and its mirror become tabu until iteration it + t
                tabu_set = (g == r / ROWS && b == (s >> 2)) || (g == s / ROWS && b == (r >> 2));
                if (g == r / ROWS && b == (s >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (j == jr && e == es) ut[j][e] = until;
                }
                if (g == s / ROWS && b == (r >> 2)) {
#pragma unroll
                    for (int j = 0; j < ROWS; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (j == js && e == er) ut[j][e] = until;
                }
            }
            if (boundary) {
                // padding slots back to BIG; the tests run on opaque copies of the tile
                // origin so that they are made here rather than kept as one mask per
                // slot through the whole loop (scalar registers the loop needs)
                int pu = u0, pv = v0;
                asm volatile("" : "+v"(pu), "+v"(pv));
#pragma unroll
                for (int j = 0; j < ROWS; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (pu + j >= n || pv + e >= n) dl[j][e] = NOMOVE;
            }
            return tabu_set;
        };
        if (!STREAM) {
            if (active) move_tile(dl, ut, g, b, boundary);
        } else {
            // each pass: load, update, find the lane's candidate for the next iteration
            // (it + 1, with cur and best after this move), store
            const int thr = aspiration();
            sel = NO_MOVE;
            for (int q = 0; q < npass; ++q) {
                const int tix = t + q * L;
                if (tix >= a.ntiles) break;
                int tg, tb;
                tile_of(tix, tg, tb);
                int d[ROWS][4], u_[UTR][4];
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    const int4 x = a.tile_d[tile_addr(q, j)];
                    d[j][0] = x.x; d[j][1] = x.y; d[j][2] = x.z; d[j][3] = x.w;
                    if (TABU && !CTB) {
                        const int4 y = a.tile_u[tile_addr(q, j)];
                        u_[j][0] = y.x; u_[j][1] = y.y; u_[j][2] = y.z; u_[j][3] = y.w;
                    }
                }
                const bool changed = move_tile(d, u_, tg, tb, tix >= a.ninterior);
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    a.tile_d[tile_addr(q, j)] = make_int4(d[j][0], d[j][1], d[j][2], d[j][3]);
                    if (TABU && !CTB && changed)
                        a.tile_u[tile_addr(q, j)] = make_int4(u_[j][0], u_[j][1], u_[j][2], u_[j][3]);
                }
                const long long c = CTB ? tile_min_bits(d, tbits[tg * nbw + tb], tg * ROWS, tb * TILE_COLS, thr)
                                        : tile_min(d, u_, tg * ROWS, tb * TILE_COLS, it + 1, thr);
                sel = c < sel ? c : sel;
            }
        }
        if (TABU && ++tpos == L) tpos = 0;
        if (TABU) ++it; else ++steps;
    }

    // ---- results
    __syncthreads();
    const int moves = TABU ? it - 1 : steps;
    const bool finished = st == nullptr || !TABU || stopped || it > a.iters;
    if (st != nullptr) {
        // save the search so a later run resumes it exactly where it stopped (opaque
        // copies of the tile origin: the slot indices are recomputed here rather than
        // kept live through the search from the load above)
        int su0 = u0, sv0 = v0;
        asm volatile("" : "+v"(su0), "+v"(sv0));
        if (!STREAM && !finished)
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = su0 + j, v = sv0 + e;
                if (active && u < v && v < n) {
                    const long long ix = pidx(n, u, v);
                    a.st_du[ix] = make_int2(PS ? dl[j][e] >> KSB : dl[j][e], TABU ? ut[j][e] : 0);
                }
            }
        for (int u = t; u < n; u += L) {
            a.st_perm[u] = perm[u];
            a.st_bestp[u] = bestp[u];
        }
        if (FREQ && a.st_mark)
            for (int u = t; u < n; u += L) a.st_mark[u] = s_mark[u];
        if (t == 0) {
            st->cur = cur;
            st->best = best;
            st->it = it;
            st->moves = moves;
            st->done = finished ? 1 : 0;
            st->last_imp = last_imp;
        }
    }
    if (finished) {
        const int *res = TABU ? bestp : perm;
        for (int u = t; u < n; u += L) a.perm_out[u] = res[u];
        if (t == 0) {
            *a.cost_out = TABU ? best : cur;
            if (a.steps_out) *a.steps_out = moves;
        }
    }
    __syncthreads();
}

// The search body for both symmetric and general instances (one uniform branch).
// CT: the compact tabu state (wide streamed tabu searches without the frequency memory,
// run whole): 0 never, 1 when the tenures fit its ring (a uniform branch), 2 always (the
// caller checked a.hi < TABU_RING).
template <int ROWS, bool TABU, int MAXT, bool RESUME, bool STREAM, bool NARROW, bool FREQ = false,
          bool GGLOB = false, int CT = 0>
__device__ __attribute__((always_inline)) void search_body(const Item &a, unsigned char *sm) {
    if constexpr (TABU && STREAM && GGLOB && !FREQ && !RESUME && CT > 0) {
        if (CT == 2 || a.hi < TABU_RING) {
            if (a.sym)
                search_body_t<ROWS, TABU, MAXT, RESUME, STREAM, true, NARROW, FREQ, GGLOB, true>(a, sm);
            else
                search_body_t<ROWS, TABU, MAXT, RESUME, STREAM, false, NARROW, FREQ, GGLOB, true>(a, sm);
            return;
        }
        if constexpr (CT == 2) return;
    }
    if (a.sym)
        search_body_t<ROWS, TABU, MAXT, RESUME, STREAM, true, NARROW, FREQ, GGLOB>(a, sm);
    else
        search_body_t<ROWS, TABU, MAXT, RESUME, STREAM, false, NARROW, FREQ, GGLOB>(a, sm);
}

// One search per workgroup: block b runs search job0 + b of the launch.
template <int ROWS, bool TABU, bool FREQ = false>
__global__ void __launch_bounds__(max_lanes<ROWS>())
__attribute__((amdgpu_waves_per_eu(!TABU && ROWS <= 8 ? 4 : 1))) search_kernel(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const int job = a.job0 + blockIdx.x;
    Item it{};
    it.mats = a.mats;
    it.tiles = a.tiles;
    it.table = a.table + (size_t)job * a.m;
    it.perm_in = a.perms_in + (size_t)job * a.n;
    it.perm_out = a.perm_out + (size_t)job * a.n;
    it.cost_out = a.cost_out + job;
    it.steps_out = a.steps_out ? a.steps_out + job : nullptr;
    it.freq = FREQ ? a.freq + (size_t)job * a.m : nullptr;
    it.div = FREQ ? a.div : 0;
    it.attr = FREQ ? a.attr : 0;
    it.uloc = FREQ && a.uloc ? a.uloc + (size_t)job * a.n * a.n : nullptr;
    it.trace = FREQ && a.trace ? a.trace + (size_t)job * a.trace_cap * 4 : nullptr;
    it.trace_cap = FREQ ? a.trace_cap : 0;
    it.st = nullptr;
    it.n = a.n;
    it.m = a.m;
    it.sym = a.sym;
    it.ntiles = a.ntiles;
    it.ninterior = a.ninterior;
    it.rows = ROWS;
    it.iters = a.iters;
    it.lo = a.lo;
    it.hi = a.hi;
    it.seed = a.seed;
    it.start_id = a.start_base + job;
    search_body<ROWS, TABU, max_tasks<ROWS>(), false, false,
                TABU ? (ROWS <= 2 || (FREQ && ROWS <= 4)) : ROWS == 8, FREQ>(it, sm);
}

// The batched launch, one kernel per tile shape: block i runs items[i] as one tabu
// search (items come sorted by decreasing work, and the hardware hands blocks to compute
// units in index order as they free up, so the longest searches start first).  Tiles of
// 2 and 4 rows ask for four waves per SIMD (at most 128 VGPRs, row dot products in
// 16-byte steps), so two searches share a compute unit and hide each other's latency;
// a 768-lane search (three waves per SIMD) then leaves a wave slot and its registers on
// every SIMD for a small search of another variant.  8-row and streamed tiles need more
// registers and run one search per compute unit.  (A persistent loop over a work queue
// inside one block was tried: keeping its state live made the register tiles spill.)
template <int ROWS, int LANES, int MAXT, bool STREAM, bool WIDE = false>
__global__ void __launch_bounds__(LANES) __attribute__((amdgpu_waves_per_eu(ROWS <= 4 ? 4 : 2)))
batch_group_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char sm[];
    Item it = b.items[blockIdx.x];
    it.perm_in = b.perms + it.perm_off;
    it.perm_out = b.perms + it.perm_off;
    it.cost_out = b.best + it.out_off;
    it.steps_out = b.done ? b.done + it.out_off : nullptr;
    it.table = b.table + it.table_off;
    if (STREAM) {
        it.tile_d = b.tile_work + it.tile_off;
        it.tile_u = it.tile_d + stream_tile_int4(it.ntiles) / 2;
    }
    if constexpr (WIDE) {
        search_body<STREAM_ROWS, true, WIDE_MAXT, false, true, false, false, true, 1>(it, sm);
    } else {
        search_body<ROWS, true, MAXT, false, STREAM, ROWS <= 4>(it, sm);
    }
}

// The batched launch of plans whose searches keep the frequency memory (and may use the
// diversification move or a unit attribute): one kernel for every tile shape, 512
// lanes, the shape taken from the item; the items' freq and uloc pointers are absolute.
__global__ void __launch_bounds__(BATCH_LANES) batch_freq_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char sm[];
    Item it = b.items[blockIdx.x];
    it.perm_in = b.perms + it.perm_off;
    it.perm_out = b.perms + it.perm_off;
    it.cost_out = b.best + it.out_off;
    it.steps_out = b.done ? b.done + it.out_off : nullptr;
    it.table = b.table + it.table_off;
    constexpr int T = 1024 / BATCH_LANES;
    if (it.stream) {
        it.tile_d = b.tile_work + it.tile_off;
        it.tile_u = it.tile_d + stream_tile_int4(it.ntiles) / 2;
        search_body<STREAM_ROWS, true, T, false, true, false, true>(it, sm);
        return;
    }
    switch (it.rows) {
        case 2: search_body<2, true, T, false, false, false, true>(it, sm); break;
        case 4: search_body<4, true, T, false, false, false, true>(it, sm); break;
        default: search_body<8, true, T, false, false, false, true>(it, sm); break;
    }
}

// Chunked runs: block i runs one chunk of items[i] (absolute pointers, st != null).
__global__ void __launch_bounds__(BATCH_LANES) resume_kernel(const Item *items) {
    extern __shared__ __align__(16) unsigned char sm[];
    const Item it = items[blockIdx.x];
    if (it.stream) {
        search_body<STREAM_ROWS, true, 1024 / BATCH_LANES, true, true, true>(it, sm);
        return;
    }
    switch (it.rows) {
        case 2: search_body<2, true, 1024 / BATCH_LANES, true, false, true>(it, sm); break;
        case 4: search_body<4, true, 1024 / BATCH_LANES, true, false, true>(it, sm); break;
        default: search_body<8, true, 1024 / BATCH_LANES, true, false, true>(it, sm); break;
    }
}

// Chunked runs of searches that keep the frequency memory: block i runs one chunk of
// items[i] (tiles of 2, 4, 8 rows or the streamed form, n up to WIDE_N).
__global__ void __launch_bounds__(BATCH_LANES) resume_freq_kernel(const Item *items) {
    extern __shared__ __align__(16) unsigned char sm[];
    const Item it = items[blockIdx.x];
    constexpr int T = 1024 / BATCH_LANES;
    if (it.stream) {
        search_body<STREAM_ROWS, true, T, true, true, false, true>(it, sm);
        return;
    }
    switch (it.rows) {
        case 2: search_body<2, true, T, true, false, false, true>(it, sm); break;
        case 4: search_body<4, true, T, true, false, false, true>(it, sm); break;
        default: search_body<8, true, T, true, false, false, true>(it, sm); break;
    }
}

// Chunked runs of searches above WIDE_N: block i runs one chunk of items[i] (the wide
// streamed form).
__global__ void __launch_bounds__(BATCH_LANES) resume_wide_kernel(const Item *items) {
    extern __shared__ __align__(16) unsigned char sm[];
    const Item it = items[blockIdx.x];
    search_body<STREAM_ROWS, true, WIDE_MAXT, true, true, false, false, true>(it, sm);
}

// Streamed search, one per workgroup: block b runs search job0 + b of the launch.  WIDE
// (n above WIDE_N): G and G^T in global scratch, up to four (index, family) tasks a lane.
// CT (wide tabu searches without the frequency memory): the compact tabu state, for
// tenures below TABU_RING
template <bool TABU, bool FREQ = false, bool WIDE = false, bool CT = false>
__global__ void __launch_bounds__(BATCH_LANES) stream_kernel(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const int job = a.job0 + blockIdx.x;
    Item it{};
    it.mats = a.mats;
    it.tiles = a.tiles;
    it.table = a.table + (size_t)job * a.m;
    it.perm_in = a.perms_in + (size_t)job * a.n;
    it.perm_out = a.perm_out + (size_t)job * a.n;
    it.cost_out = a.cost_out + job;
    it.steps_out = a.steps_out ? a.steps_out + job : nullptr;
    it.freq = FREQ ? a.freq + (size_t)job * a.m : nullptr;
    it.div = FREQ ? a.div : 0;
    it.attr = FREQ ? a.attr : 0;
    it.uloc = FREQ && a.uloc ? a.uloc + (size_t)job * a.n * a.n : nullptr;
    it.trace = FREQ && a.trace ? a.trace + (size_t)job * a.trace_cap * 4 : nullptr;
    it.trace_cap = FREQ ? a.trace_cap : 0;
    it.n = a.n;
    it.m = a.m;
    it.sym = a.sym;
    it.ntiles = a.ntiles;
    it.ninterior = a.ninterior;
    it.rows = STREAM_ROWS;
    it.iters = a.iters;
    it.lo = a.lo;
    it.hi = a.hi;
    it.seed = a.seed;
    it.start_id = a.start_base + job;
    it.stream = 1;
    it.tile_d = a.tile_work + (size_t)blockIdx.x * a.tile_stride;
    it.tile_u = it.tile_d + a.tile_stride / 2;
    if constexpr (WIDE) {
        search_body<STREAM_ROWS, TABU, WIDE_MAXT, false, true, false, FREQ, true, CT ? 2 : 0>(it, sm);
    } else {
        search_body<STREAM_ROWS, TABU, 1024 / BATCH_LANES, false, true, false, FREQ>(it, sm);
    }
}

template <int ROWS, bool TABU, bool FREQ = false>
hipError_t launch_one(const SearchArgs &a, int grid, int lanes, size_t smem, hipStream_t st) {
    hipLaunchKernelGGL((search_kernel<ROWS, TABU, FREQ>), dim3(grid), dim3(lanes), smem, st, a);
    return report(hipGetLastError(), "kernel launch");
}

}  // namespace

int search_max_lanes(int rows) {
    return rows <= 2 ? max_lanes<2>() : (rows == 4 ? max_lanes<4>() : (rows <= 8 ? max_lanes<8>() : max_lanes<16>()));
}

namespace {
template <int ROWS, bool TABU>
int blocks_one(int lanes, size_t smem) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search_kernel<ROWS, TABU>, lanes, smem) != hipSuccess)
        return 0;
    return nb;
}
}  // namespace

int search_blocks_per_cu(int n, int rows, bool tabu, int lanes, int sym) {
    const size_t smem = search_smem_bytes(n, rows, lanes, sym);
    switch (rows * 2 + (tabu ? 1 : 0)) {
        case 2: return blocks_one<1, false>(lanes, smem);
        case 3: return blocks_one<1, true>(lanes, smem);
        case 4: return blocks_one<2, false>(lanes, smem);
        case 5: return blocks_one<2, true>(lanes, smem);
        case 8: return blocks_one<4, false>(lanes, smem);
        case 9: return blocks_one<4, true>(lanes, smem);
        case 16: return blocks_one<8, false>(lanes, smem);
        case 17: return blocks_one<8, true>(lanes, smem);
        case 32: return blocks_one<16, false>(lanes, smem);
        case 33: return blocks_one<16, true>(lanes, smem);
        default: return 0;
    }
}

// Block size for a tile shape: at least one lane per tile; one lane per (index, family)
// task when the workgroup limit allows, else up to MAXT tasks per lane.  Returns 0 when
// the shape cannot serve n.
int search_lanes(int n, int rows, int ntiles, int sym) {
    const int maxl = search_max_lanes(rows);
    const int tasks = families(sym) * n;
    int lanes = (ntiles + 63) / 64 * 64;
    if (lanes < 64) lanes = 64;
    if (lanes > maxl) return 0;
    const int want = (tasks + 63) / 64 * 64;
    if (want > lanes) lanes = want < maxl ? want : maxl;
    const int maxt = 1024 / maxl;
    const int need = ((tasks + maxt - 1) / maxt + 63) / 64 * 64;
    if (need > lanes) lanes = need;
    return lanes <= maxl ? lanes : 0;
}

int batch_variant(int n, int rows, bool streamed, int ntiles, int sym) {
    if (streamed) return n > WIDE_N ? BV_WIDE : BV_STREAM;
    // lanes a one-task workgroup needs: one per tile and one per (index, family) task
    // (the 512-lane kernels of 2 and 4 rows carry one task a lane: at most 512 tiles of
    // those shapes means n below 128, 4 n < 512 tasks; the checks keep it so)
    const int need = ntiles > families(sym) * n ? ntiles : families(sym) * n;
    if (rows == 2) return need <= 128 ? BV_R2_128 : (need <= 256 ? BV_R2_256 : (need <= BATCH_LANES ? BV_R2 : -1));
    if (rows == 4) return need <= 256 ? BV_R4_256 : (need <= BATCH_LANES ? BV_R4 : BV_R4_768);
    return BV_R8;
}

int batch_variant_lanes(int variant) {
    if (variant == BV_R4_768) return 768;
    return variant == BV_R2_128 ? 128 : (variant == BV_R2_256 || variant == BV_R4_256 ? 256 : BATCH_LANES);
}

int batch_shape_ok_wide(int n, int rows, int ntiles, int sym) {
    return batch_shape_ok(n, rows, ntiles, sym) || (rows == 4 && ntiles <= 768 && families(sym) * n <= 768) ? 1 : 0;
}

int batch_shape_ok(int n, int rows, int ntiles, int sym) {
    return rows <= 8 && ntiles <= BATCH_LANES && families(sym) * n <= BATCH_LANES * (1024 / BATCH_LANES) ? 1 : 0;
}

hipError_t launch_batch_group(int variant, const BatchArgs &b, size_t smem, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    constexpr int L = BATCH_LANES, T = 1024 / BATCH_LANES;
    switch (variant) {
        case BV_R2: hipLaunchKernelGGL((batch_group_kernel<2, L, 1, false>), dim3(b.count), dim3(L), smem, st, b); break;
        case BV_R4: hipLaunchKernelGGL((batch_group_kernel<4, L, 1, false>), dim3(b.count), dim3(L), smem, st, b); break;
        case BV_R8: hipLaunchKernelGGL((batch_group_kernel<8, L, T, false>), dim3(b.count), dim3(L), smem, st, b); break;
        case BV_R2_128:
            hipLaunchKernelGGL((batch_group_kernel<2, 128, 1, false>), dim3(b.count), dim3(128), smem, st, b);
            break;
        case BV_R2_256:
            hipLaunchKernelGGL((batch_group_kernel<2, 256, 1, false>), dim3(b.count), dim3(256), smem, st, b);
            break;
        case BV_R4_256:
            hipLaunchKernelGGL((batch_group_kernel<4, 256, 1, false>), dim3(b.count), dim3(256), smem, st, b);
            break;
        case BV_R4_768:
            hipLaunchKernelGGL((batch_group_kernel<4, 768, 1, false>), dim3(b.count), dim3(768), smem, st, b);
            break;
        case BV_STREAM:
            hipLaunchKernelGGL((batch_group_kernel<STREAM_ROWS, L, T, true>), dim3(b.count), dim3(L), smem, st, b);
            break;
        case BV_WIDE:
            hipLaunchKernelGGL((batch_group_kernel<STREAM_ROWS, L, WIDE_MAXT, true, true>), dim3(b.count), dim3(L),
                               smem, st, b);
            break;
        default: return hipErrorInvalidValue;
    }
    return report(hipGetLastError(), "batch kernel launch");
}


hipError_t launch_batch_freq(const BatchArgs &b, size_t smem, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_freq_kernel, dim3(b.count), dim3(BATCH_LANES), smem, st, b);
    return report(hipGetLastError(), "batch kernel launch");
}

size_t freq_static_lds() {
    static const size_t bytes = [] {
        size_t m = 0;
        hipFuncAttributes fa{};
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(batch_freq_kernel)) == hipSuccess)
            m = fa.sharedSizeBytes > m ? fa.sharedSizeBytes : m;
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(resume_freq_kernel)) == hipSuccess)
            m = fa.sharedSizeBytes > m ? fa.sharedSizeBytes : m;
        return m;
    }();
    return bytes;
}

hipError_t launch_resume_freq(const Item *d_items, int count, size_t smem, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(resume_freq_kernel, dim3(count), dim3(BATCH_LANES), smem, st, d_items);
    return report(hipGetLastError(), "resume kernel launch");
}

hipError_t launch_resume_wide(const Item *d_items, int count, size_t smem, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(resume_wide_kernel, dim3(count), dim3(BATCH_LANES), smem, st, d_items);
    return report(hipGetLastError(), "resume kernel launch");
}

hipError_t launch_resume(const Item *d_items, int count, size_t smem, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(resume_kernel, dim3(count), dim3(BATCH_LANES), smem, st, d_items);
    return report(hipGetLastError(), "resume kernel launch");
}

size_t stream_smem_bytes(int n, int sym) {
    return (size_t)smem_plan(n, padded_n(n, STREAM_ROWS), BATCH_LANES, sym, true, n > WIDE_N).total;
}

int stream_shape_ok(int n, int sym, size_t max_smem) {
    const int tasks = n <= WIDE_N ? 1024 : (n <= WIDE_MAXN ? BATCH_LANES * WIDE_MAXT : 0);
    return families(sym) * n <= tasks && stream_smem_bytes(n, sym) <= max_smem ? 1 : 0;
}

// grid = searches in this launch; a.tile_work holds grid * a.tile_stride int4.
hipError_t launch_stream(bool tabu, const SearchArgs &a, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    const size_t smem = stream_smem_bytes(a.n, a.sym);
    if (a.n > WIDE_N) {   // the wide form
        if (tabu && a.freq)
            hipLaunchKernelGGL((stream_kernel<true, true, true>), dim3(grid), dim3(BATCH_LANES), smem, st, a);
        else if (tabu && a.hi < TABU_RING)
            hipLaunchKernelGGL((stream_kernel<true, false, true, true>), dim3(grid), dim3(BATCH_LANES), smem, st, a);
        else if (tabu)
            hipLaunchKernelGGL((stream_kernel<true, false, true>), dim3(grid), dim3(BATCH_LANES), smem, st, a);
        else
            hipLaunchKernelGGL((stream_kernel<false, false, true>), dim3(grid), dim3(BATCH_LANES), smem, st, a);
    } else if (tabu && a.freq)
        hipLaunchKernelGGL((stream_kernel<true, true>), dim3(grid), dim3(BATCH_LANES), smem, st, a);
    else if (tabu)
        hipLaunchKernelGGL(stream_kernel<true>, dim3(grid), dim3(BATCH_LANES), smem, st, a);
    else
        hipLaunchKernelGGL(stream_kernel<false>, dim3(grid), dim3(BATCH_LANES), smem, st, a);
    return report(hipGetLastError(), "stream kernel launch");
}

size_t search_smem_bytes(int n, int rows, int lanes, int sym) {
    return (size_t)smem_plan(n, padded_n(n, rows), lanes, sym).total;
}

hipError_t launch_search(int rows, bool tabu, const SearchArgs &a, int grid, int lanes, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    const size_t smem = search_smem_bytes(a.n, rows, lanes, a.sym);
    if (tabu && a.freq) {   // the frequency memory: its own instantiations
        switch (rows) {
            case 1: return launch_one<1, true, true>(a, grid, lanes, smem, st);
            case 2: return launch_one<2, true, true>(a, grid, lanes, smem, st);
            case 4: return launch_one<4, true, true>(a, grid, lanes, smem, st);
            case 8: return launch_one<8, true, true>(a, grid, lanes, smem, st);
            case 16: return launch_one<16, true, true>(a, grid, lanes, smem, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (rows * 2 + (tabu ? 1 : 0)) {
        case 2: return launch_one<1, false>(a, grid, lanes, smem, st);
        case 3: return launch_one<1, true>(a, grid, lanes, smem, st);
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
