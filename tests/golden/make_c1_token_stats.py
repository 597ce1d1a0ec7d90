"""Writes c1_token_stats.txt: the per-token row counts and spreads of the
10M-row workload (30,522 Zipf(1.0) token ids, four sub-centres per token),
computed by the oracle from the seeded generator -- the statistics the budget
of Sect. 2.1 takes as input.

Only tokens with at least 256 rows are written: they are the budget's active
tokens, the only ones whose spread enters it (tail tokens get one or two
centroids from their count alone).  Spreads are written with repr(), which
reads back to the same float64.

Run from the repository root: ``python tests/golden/make_c1_token_stats.py``
(under a minute and about 12 GB of host memory)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_token_stats.txt")
ACTIVE_MIN = 256


def main():
    w = datagen.WORKLOADS["c1"]
    x, tok = datagen.make(w)
    perm, seg_off, counts = oracle.group_by_token(tok, w.vocab)
    del tok
    xs = x[perm]
    del x, perm
    spread = oracle.spreads(xs, seg_off)
    with open(OUT, "w") as f:
        f.write("# Per-token statistics of the 10M-row workload (30,522 Zipf(1.0) ids, seed 0), written by\n")
        f.write("# tests/golden/make_c1_token_stats.py from the oracle (group_by_token, spreads).\n")
        f.write(f"# tokens with at least {ACTIVE_MIN} rows: token id, rows n_j, spread s_j (float64 repr)\n")
        for j in np.nonzero(counts >= ACTIVE_MIN)[0]:
            f.write(f"{j} {counts[j]} {float(spread[j])!r}\n")


if __name__ == "__main__":
    main()
