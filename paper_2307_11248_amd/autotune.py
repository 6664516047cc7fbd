"""Tile-shape autotuner per n, with a JSON cache.

The paper picks its thread configuration per instance size by a search over thread
counts and block sizes (Sec. 5.2, Eq. (3)).  Here the free parameter is the tile shape
of the search kernels (rows of the register tile each lane owns), and it is chosen by
measurement: ``qap_tune_tile_rows`` times every shape that fits n on the device and keeps
the fastest.  The time depends on n, on whether F and D are both symmetric, and on the
algorithm, not on the matrix values (a tabu search does the same work every iteration),
so one measurement serves every instance with the same key, and the cache keeps it
across processes.  The key also names the GPU architecture and a digest of the built
library, so a rebuilt kernel is tuned again.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

from . import qap

# Relative time difference below which two tile shapes of a batched search count as
# equally fast, and the size of the timing runs of batched shapes.
BATCH_MARGIN = 0.03
BATCH_STARTS, BATCH_ITERS = 4096, 150

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "paper_2307_11248_amd", "tile_rows.json")


def _lib_digest() -> str:
    h = hashlib.sha1()
    with open(qap.LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:12]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


class TileCache:
    """Tuned tile rows per (architecture, library, algorithm, n, symmetric)."""

    def __init__(self, path: str | None = None, k: int = 256, iters: int = 500):
        self.path = path or os.environ.get("QAP_TUNE_CACHE", DEFAULT_PATH)
        self.k, self.iters = k, iters
        self.prefix = "%s|%s" % (_arch(), _lib_digest())
        self.entries = {}
        self.tuned = 0            # shapes measured by this object (cache misses)
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.entries = json.load(f)

    def key(self, algo: str, n: int, sym: bool) -> str:
        return "%s|%s|%d|%s" % (self.prefix, algo, n, "sym" if sym else "asym")

    def apply(self, h: "qap.Handle", algo: str) -> int:
        """Set the tuned shape on handle h (measuring it first on a cache miss); returns rows."""
        k = self.key(algo, h.n, h.sym)
        rows = self.entries.get(k, {}).get("rows")
        if rows is not None:
            try:
                h.set_tile_rows(algo, rows)
                return rows
            except qap.QapError:
                pass                      # the cached shape no longer fits: measure again
        # the batched kernels run several searches per compute unit: time enough searches
        # to fill the device several times over (4096, about 16 a compute unit, more than
        # fit at once), so the choice reflects throughput, not one search's latency
        if algo == "batch":
            starts, iters = max(self.k, BATCH_STARTS), BATCH_ITERS
        else:
            starts, iters = self.k, self.iters
        rows, times = h.tune_tile_rows(algo, starts, iters)
        if algo == "batch" and times:
            # shapes within BATCH_MARGIN of the fastest time within noise of each other; take
            # the largest register tile among them (fewer lanes per search, so more searches
            # share a compute unit in a mixed batch), which keeps the choice stable
            fastest = min(times.values())
            near = [r for r, t in times.items() if r > 0 and t <= fastest * (1 + BATCH_MARGIN)]
            if near and max(near) != rows:
                rows = max(near)
                h.set_tile_rows(algo, rows)
        self.entries[k] = {"rows": rows, "ms": {str(r): t for r, t in times.items()}}
        self.tuned += 1
        return rows

    def apply_all(self, handles, algo: str) -> list:
        """Tune one handle per distinct (n, symmetric) and give its shape to the rest."""
        chosen, out = {}, []
        for h in handles:
            kk = (h.n, h.sym)
            if kk not in chosen:
                chosen[kk] = self.apply(h, algo)
            else:
                h.set_tile_rows(algo, chosen[kk])
            out.append(chosen[kk])
        return out

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tile_rows.")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
