"""Write the oracle's C_l for the full-size T/E/lensing workload (l = 2..2500,
4000 log-k on [1e-4, 0.5], 3000 tau) at sampled multipoles.

Calls only the CPU oracle (and the seeded input generator).  Output:
``c2_cl_oracle.txt`` with one line per sampled l: ``l TT EE TE PP`` (repr floats).
Run from the repository root: ``python tests/golden/make_golden.py``.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_25110_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_cl_oracle.txt")


def sampled_ells(lmin, lmax):
    ls = set(range(lmin, min(lmin + 48, lmax + 1)))
    ls.update(range(lmin, lmax + 1, 7))
    ls.update(range(max(lmin, lmax - 8), lmax + 1))
    return sorted(ls)


def main():
    w = inputs.config("C2")
    t = time.time()
    d = oracle.project(w.lmin, w.lmax, w.k, w.tau, w.tau0, w.w_tau, w.S)
    c = oracle.cl(d, w.w_lnk, w.Pk, w.pairs)
    ls = sampled_ells(w.lmin, w.lmax)
    with open(OUT, "w") as f:
        f.write("# oracle C_l, workload C2 (%s); columns: l %s\n"
                % (inputs.DESCRIPTIONS["C2"], " ".join(w.pair_names)))
        f.write("# written by tests/golden/make_golden.py with %d oracle threads in %.0f s\n"
                % (oracle.num_threads(), time.time() - t))
        for l in ls:
            f.write("%d %s\n" % (l, " ".join(repr(float(v)) for v in c[:, l - w.lmin])))
    print("wrote", OUT, len(ls), "rows")


if __name__ == "__main__":
    main()
