"""Write the full-size expected results that the GPU parity tests compare with.

Run from the repository root:  python tests/golden/make_full_fixtures.py [dense|t40|batch ...]

Every expected value here comes from the CPU oracle (oracle/oracle.cpp through
oracle.cpp), run to completion on the seeded synthetic workloads of gen/; nothing
is taken from the GPU library.  Outputs:

  full_dense_planted_1M.npz   1,000,000 x 4,096 dense planted workload, minsup 10,000
  full_quest_t40_1M.npz       1,000,000 x 2,000 T40-style workload, minsup 5,000
      lengths u8[F], items u16[sum], supports u32[F] (canonical order), the
      oracle's candidate count, and SHA-256 digests of the input CSR so that a
      change of the generator is reported as such and not as a mining error;
  full_batch_256.json         the 256 Quest-style databases of the batched
      workload: per database the input digest, the result's set/item counts,
      candidates, and the SHA-256 of its canonical arrays (offsets as little-endian
      u64, items and supports as little-endian u32) -- 357k itemsets in all,
      compared as digests to keep the fixture small.

The dense and T40 runs take about a minute and three minutes on eight cores.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
from oracle import cpp as ocpp  # noqa: E402

FULL = {"dense": (3, "full_dense_planted_1M.npz"), "t40": (5, "full_quest_t40_1M.npz")}
BATCH = "full_batch_256.json"


def input_digest(db) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(db.row_ptr, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(db.col_idx, dtype="<u4").tobytes())
    h.update(f"{db.n},{db.m},{db.minsup}".encode())
    return h.hexdigest()


def result_digest(offs, items, supp) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offs, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(items, dtype="<u4").tobytes())
    h.update(np.ascontiguousarray(supp, dtype="<u4").tobytes())
    return h.hexdigest()


def write_full(which: str) -> None:
    k, name = FULL[which]
    db = gen.make_config(k)
    t0 = time.time()
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    offs, items, supp, cands = o.mine_arrays(db.minsup)
    lens = np.diff(offs.astype(np.int64))
    assert lens.max() < 256 and db.m <= 65536
    np.savez_compressed(os.path.join(HERE, name), lengths=lens.astype(np.uint8),
                        items=items.astype(np.uint16), supports=supp.astype(np.uint32),
                        candidates=np.array([cands], dtype=np.uint64),
                        input_sha256=np.array([input_digest(db)]),
                        result_sha256=np.array([result_digest(offs, items, supp)]))
    print(f"{name}: {len(supp)} sets, {cands} candidates, {time.time() - t0:.1f} s", flush=True)


def write_batch() -> None:
    dbs = gen.batch_dbs(256)
    t0 = time.time()
    rows = []
    for k, d in enumerate(dbs):
        o = ocpp.OracleDb(d.row_ptr, d.col_idx, d.n, d.m)
        offs, items, supp, cands = o.mine_arrays(d.minsup)
        rows.append({"k": k, "name": d.name, "n": int(d.n), "m": int(d.m), "minsup": int(d.minsup),
                     "input_sha256": input_digest(d), "sets": int(len(supp)),
                     "items": int(len(items)), "candidates": int(cands),
                     "result_sha256": result_digest(offs, items, supp)})
    with open(os.path.join(HERE, BATCH), "w") as f:
        json.dump({"workload": "256 Quest-style databases (gen.batch_dbs(256))", "databases": rows},
                  f, indent=0)
        f.write("\n")
    print(f"{BATCH}: {sum(r['sets'] for r in rows)} sets, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["dense", "t40", "batch"]
    for w in todo:
        write_batch() if w == "batch" else write_full(w)
