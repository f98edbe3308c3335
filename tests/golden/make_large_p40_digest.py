"""Write large_p40_oracle_digest.json: a digest of the CPU oracle's RT-DetMCD
fit of the 10,000,000 x 40 stream-like workload (1,024 blocks of 9,765 rows,
640 remainder rows), against which the GPU fit of the same seeded data is
compared.  Calls only oracle/ and synthdata/ (the seeded generator); takes
several minutes and about 20 GB of memory on one core.

    python tests/golden/make_large_p40_digest.py
"""
from __future__ import annotations

import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synthdata  # noqa: E402

N_CHUNKS = 1024
SAMPLE_ROWS = 4096


def crc(a: np.ndarray) -> int:
    return int(zlib.crc32(np.ascontiguousarray(a).tobytes()))


def main() -> None:
    t0 = time.time()
    ds = synthdata.workload_large_p40()
    ref = oracle.fit(ds.X, n_chunks=N_CHUNKS)
    H = ref.hsubset.astype(np.int32)
    flagged = np.nonzero(ref.outlier)[0].astype(np.int64)
    rows = np.random.default_rng(20).choice(ds.X.shape[0], SAMPLE_ROWS, replace=False)
    rows.sort()
    out = {
        "workload": "synthdata.workload_large_p40(), oracle.fit(X, n_chunks=1024)",
        "q": ref.q, "m": ref.m, "h": ref.h,
        "loc": ref.loc.tolist(), "scale": ref.scale.tolist(),
        "block_status": ref.chunk_status.tolist(),
        "block_start": ref.chunk_start.tolist(),
        "block_iters": ref.chunk_iters.tolist(),
        "hsubset_crc32": [crc(H[b]) for b in range(ref.q)],
        "hsubset_sum": [int(H[b].astype(np.int64).sum()) for b in range(ref.q)],
        "mu_raw": ref.mu_raw.tolist(), "sigma_raw": ref.sigma_raw.tolist(),
        "mu": ref.mu.tolist(), "sigma": ref.sigma.tolist(),
        "logdet_raw": ref.logdet_raw, "logdet_rew": ref.logdet_rew,
        "n_w": int(ref.n_w),
        "rew_mask_crc32": crc(ref.rew_mask.astype(np.uint8)),
        "n_flagged": int(flagged.size),
        "flagged_crc32": crc(flagged),
        "dist_rows": rows.tolist(),
        "dist_at_rows": ref.dist[rows].tolist(),
        "kept_blocks": [int(b) for b in ref.diag["keep"]],
        "seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, "large_p40_oracle_digest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} in {out['seconds']} s")


if __name__ == "__main__":
    main()
