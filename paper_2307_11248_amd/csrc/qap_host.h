// qap_host.h -- host helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

struct qap_ctx;

namespace qaph {

// Tile heights of the search kernels.
constexpr int kShapes = 5;   // register tile shapes: rows 1, 2, 4, 8, 16
extern const int kRowsChoices[kShapes];

// Tiles of `rows` x 4 that hold at least one move (u < v), interior tiles first; each
// entry is g | b << 16 (row group g, column block b).
std::vector<int32_t> enumerate_tiles(int n, int rows, int *ninterior);

// Range-check F and D (entries in [0, 255]) and pack [F | F^T | D | D^T] as u8 rows of
// row_stride(n) bytes; *sym = 1 when F and D are both symmetric.  QAP_OK or QAP_E_RANGE.
int pack_instance(const int32_t *F, const int32_t *D, int n, std::vector<uint8_t> &pack, int *sym);

// Map a HIP status to a QAP code (QAP_VERBOSE in the environment also reports it).
int dev_err_at(hipError_t e, const char *where);
#define dev_err(e) ::qaph::dev_err_at((e), __func__)

// Whether each of the k rows of perms is a permutation of 0..n-1.
bool check_perms(const int32_t *perms, int k, int n);

// A handle's device copy of [F | F^T | D | D^T], its n, symmetry and device (for the
// server's requests on existing handles).  False for a null handle.
bool handle_view(const struct ::qap_ctx *h, const uint8_t **mats, int *n, int *sym, int *device);

// Whether a tabu run of `iters` iterations with tenures in [lo, hi] is valid: the
// iteration until which a move stays tabu, it + t <= iters + hi, must fit in int32.
inline bool tenure_args_ok(int32_t iters, int32_t lo, int32_t hi) {
    return iters >= 0 && lo >= 0 && lo <= hi && (int64_t)iters + hi < INT32_MAX;
}

}  // namespace qaph
