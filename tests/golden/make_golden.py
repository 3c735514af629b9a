"""Writes tests/golden/streams.json: frozen sign and row streams of the oracle.

Run from the repository root:  python tests/golden/make_golden.py
It calls only the oracle; the GPU parity tests compare the library's streams
with these values bit for bit.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rng  # noqa: E402

CASES = [  # (seed, n', r)
    (1, 4096, 512),
    (7, 1 << 12, 17),
    (123456789, 1 << 16, 1000),
    (2, 1 << 20, 4096),
    (0xDEADBEEFCAFEF00D, 1 << 10, 1023),
    (3, 2, 1),
]


def main():
    out = {"note": "written by tests/golden/make_golden.py from oracle.rng", "cases": []}
    for seed, n_pad, r in CASES:
        s = rng.signs(seed, n_pad)
        neg = [int(j) for j in (s < 0).nonzero()[0][:256]]
        out["cases"].append({
            "seed": seed, "n_pad": n_pad, "r": r,
            "rows_exact": [int(v) for v in rng.rows_exact(seed, n_pad, r)],
            "rows_bernoulli_head": [int(v) for v in rng.rows_bernoulli(seed, n_pad, r)[:512]],
            "rows_bernoulli_count": int(rng.rows_bernoulli(seed, n_pad, r).size),
            "neg_sign_rows_head": neg,
            "neg_sign_count": int((s < 0).sum()),
        })
    with open(os.path.join(HERE, "streams.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
