"""Writes ``rmat22_oracle.txt``: oracle N, D and EF of selected seeds of the
R-MAT scale-22, edge-factor-10 graph (the headline workload), for the
full-size parity tests.

Calls only the CPU oracle (``oracle.ef``, the plain enumeration of Eq. 1's
event sequences with Algorithm 1's multiplicities) and the seeded generator;
nothing from the GPU library. Run once (about 10 minutes on 8 host threads:
the largest hub alone is about 1.3e10 event sequences):

    python tests/golden/make_rmat22_golden.py [threads]

Seeds, in three groups (a node may sit in more than one; it is listed once):
  hub   - every node of degree > 20000 (the centres with the most clusters;
          their seeds have up to 1.3e10 sequences, far above 2^24);
  big   - 40 nodes drawn (seed 8192) from those of degree 8193..20000, the
          per-seed formulation's bitmap bin;
  strat - per degree band [0,1), [1,2), [2,4), [4,16), [16,64), [64,256),
          [256,1024), [1024,4096), [4096,16384), [16384,20001) up to 40 nodes
          drawn with seed 22, plus the three largest nodes of degree <= 20000.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2306_00606_amd import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat22_oracle.txt")


def select(deg):
    groups = {}
    for v in np.flatnonzero(deg > 20000):
        groups.setdefault(int(v), set()).add("hub")
    mid = np.flatnonzero((deg > 8192) & (deg <= 20000))
    for v in np.random.default_rng(8192).choice(mid, min(40, mid.size), replace=False):
        groups.setdefault(int(v), set()).add("big")
    rng = np.random.default_rng(22)
    bands = [0, 1, 2, 4, 16, 64, 256, 1024, 4096, 16384, 20001]
    for lo, hi in zip(bands[:-1], bands[1:]):
        idx = np.flatnonzero((deg >= lo) & (deg < hi))
        if idx.size:
            for v in rng.choice(idx, min(40, idx.size), replace=False):
                groups.setdefault(int(v), set()).add("strat")
    small = np.flatnonzero(deg <= 20000)
    for v in small[np.argsort(deg[small], kind="stable")[-3:]]:
        groups.setdefault(int(v), set()).add("strat")
    return groups


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    rp, ci = gen.rmat_22()
    deg = np.diff(rp).astype(np.int64)
    groups = select(deg)
    # largest seeds first, so the dynamic schedule balances the threads
    seeds = np.array(sorted(groups, key=lambda v: (-deg[v], v)), np.int32)
    t0 = time.perf_counter()
    N, D, E = oracle.ef(rp, ci, seeds=seeds, threads=threads)
    dt = time.perf_counter() - t0
    with open(OUT, "w") as f:
        f.write("# Oracle N, D, EF of selected seeds of R-MAT scale 22, edge factor 10\n")
        f.write("# (a=.57 b=.19 c=.19 d=.05, seed 1, id permutation seed 3; gen.rmat_22()).\n")
        f.write(f"# Written by tests/golden/make_rmat22_golden.py with the CPU oracle only\n")
        f.write(f"# ({threads} threads, {dt:.0f} s; {int(N.sum())} event sequences).\n")
        f.write("# node | degree | groups | N | D | EF (repr of the double)\n")
        for s, n_, d_, e_ in sorted(zip(seeds.tolist(), N.tolist(), D.tolist(), E.tolist())):
            f.write(f"{s} | {int(deg[s])} | {','.join(sorted(groups[s]))} | {n_} | {d_} | "
                    f"{e_!r}\n")
    print(f"wrote {len(seeds)} seeds to {OUT} in {dt:.0f} s")


if __name__ == "__main__":
    main()
