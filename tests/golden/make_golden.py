"""Write oracle_small.json: oracle results of small seeded partition tasks.

Calls only the oracle (and the seeded input generator for its inputs).  The
paper prints no worked numeric example (its demos in sec. 3.2 are described,
not measured), so these values pin the oracle against later drift and give the
GPU tests a fixed small-case expectation; they are not paper values.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402

CASES = [
    # kid, n, pid, ops
    (datagen.POLY, 1, 0, datagen.SUM | datagen.MAX),
    (datagen.POLY, 4097, 1, datagen.SUM),
    (datagen.POLY, 65536, 2, datagen.SUM | datagen.MAX),
    (datagen.FMUL, 3, 3, datagen.SUM | datagen.MAX),
    (datagen.FMUL, 100_001, 4, datagen.SUM | datagen.MAX),
    (datagen.FMUL, 262_144, 5, datagen.MAX),
    (datagen.MC_PI, 1, 6, datagen.COUNT),
    (datagen.MC_PI, 9999, 7, datagen.COUNT),
    (datagen.MC_PI, 1 << 18, 8, datagen.COUNT),
]


def compute():
    out = []
    for kid, n, pid, ops in CASES:
        p = datagen.make_part(kid, n, pid, ops=ops)
        r = oracle.run_task(kid, ops, n, p.x, p.y, seed=p.seed, pid=pid,
                            coef=p.coef, c=p.c)
        out.append({"kernel_id": kid, "n": n, "pid": pid, "ops": ops,
                    "sum": float(r.sum).hex(), "max": float(r.max).hex(),
                    "count": int(r.count)})
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_golden.py", "cases": compute()},
                  f, indent=1)
        f.write("\n")
    print("wrote", path)
