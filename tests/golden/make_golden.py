"""Writes the stored oracle values the full-size GPU parity tests compare
against.  Calls only the float64 oracle (oracle/) and the seeded coupling
generator (workloads/); nothing here touches the HIP library.

    python tests/golden/make_golden.py            # writes tests/golden/*.json

Each record holds, for one instance: the oracle's ln Z estimate, the
truncation conditioning of its build, and a few configurations drawn by the
oracle's own sampler (Philox stream of the stated seed) with their log q,
the configurations bit-packed (row-major, bit c of a row is 1 iff spin
(r, c) is +1), zlib-compressed and base64-encoded.
"""
from __future__ import annotations

import base64
import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads                                   # noqa: E402
from oracle import bmps, sampler                   # noqa: E402

# (file, family, L, config id, instance indices, chi, beta, draws, seed,
#  alternating sweep order)
RECORDS = [
    # the headline batch: instances 0 and 1 of the 256 +-J disorders of 256x256
    ("fullsize_256_chi32.json", "pmj", 256, 3, (0, 1), 32, 1.0, 3, 0x0C3, False),
    # the same instances compressed in the alternating sweep order
    ("fullsize_256_chi32_alt.json", "pmj", 256, 3, (0, 1), 32, 1.0, 3, 0x0C3, True),
    # the paper's run: +-J EA, 1024x1024, beta = 1, chi = 8
    ("paper_1024_chi8.json", "pmj", 1024, 7, (0,), 8, 1.0, 1, 0x1024, False),
]


def pack_bits(bits: np.ndarray) -> str:
    """(n, L, L) 0/1 -> zlib + base64 of the row-major packed bits."""
    raw = np.packbits(bits.astype(np.uint8), axis=-1, bitorder="little").tobytes()
    return base64.b64encode(zlib.compress(raw, 9)).decode()


def unpack_bits(text: str, n: int, L: int) -> np.ndarray:
    raw = np.frombuffer(zlib.decompress(base64.b64decode(text)), dtype=np.uint8)
    return np.unpackbits(raw.reshape(n, L, -1), axis=-1, count=L, bitorder="little").astype(np.int64)


def make(name, family, L, cfg, idx, chi, beta, draws, seed, alternate):
    out = {"family": family, "L": L, "config_id": cfg, "chi": chi, "beta": beta, "draws": draws,
           "seed": seed, "alternate": alternate, "instances": []}
    for i in idx:
        jh, jv = workloads.instance(L, family, cfg, i)
        t0 = time.time()
        dg = {}
        cache, _, logz = bmps.build_cache(beta, jh, jv, chi, dg, alternate=alternate)
        t1 = time.time()
        bits, logq, _ = sampler.sample(cache, beta, jv, draws, seed=seed, instance=i)
        print(f"{name}: instance {i} build {t1 - t1 + (t1 - t0):.0f} s, sampling {time.time() - t1:.0f} s",
              flush=True)
        out["instances"].append({"index": i, "logz": logz, "cond": float(dg.get("cond", 0.0)),
                                 "logq": [float(v) for v in logq], "bits": pack_bits(bits)})
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    only = sys.argv[1:]
    for rec in RECORDS:
        if not only or rec[0] in only:
            make(*rec)
