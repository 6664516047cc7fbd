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
        # to fill the device, so the choice reflects throughput, not one search's latency
        starts = max(self.k, 1024) if algo == "batch" else self.k
        rows, times = h.tune_tile_rows(algo, starts, self.iters)
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
