"""Write the oracle's C_l for a full-size T/E/lensing workload at sampled
multipoles: C2 (l = 2..2500, 4000 log-k on [1e-4, 0.5], 3000 tau) or C3
(l = 2..5000, 8000 log-k on [1e-4, 1], 4000 tau).

Calls only the CPU oracle (and the seeded input generator).  Output:
``c2_cl_oracle.txt`` / ``c3_cl_oracle.txt`` with one line per sampled l:
``l TT EE TE PP`` (repr floats).
``python tests/golden/make_golden.py C4`` writes ``c4_cl_oracle.txt``: the
oracle's C_l of drawn models 0 and 3 of the 256-model batch (seeded draws,
each model solved alone on its own subset of the 8000-point master k grid,
3000 tau), one line per sampled l: ``model l TT EE TE PP``.
Run from the repository root: ``python tests/golden/make_golden.py [C2|C3|C4]``.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_25110_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sampled_ells(lmin, lmax):
    ls = set(range(lmin, min(lmin + 48, lmax + 1)))
    ls.update(range(lmin, lmax + 1, 7))
    ls.update(range(max(lmin, lmax - 8), lmax + 1))
    return sorted(ls)


C4_MODELS = (0, 3)


def main_c4():
    out = os.path.join(HERE, "c4_cl_oracle.txt")
    draws = inputs.draw_models(256)
    t = time.time()
    lines = []
    for m in C4_MODELS:
        w = inputs.model_workload(draws[m])
        d = oracle.project(w.lmin, w.lmax, w.k, w.tau, w.tau0, w.w_tau, w.S)
        c = oracle.cl(d, w.w_lnk, w.Pk, w.pairs)
        for l in sampled_ells(w.lmin, w.lmax):
            lines.append("%d %d %s\n" % (m, l, " ".join(repr(float(v)) for v in c[:, l - w.lmin])))
    with open(out, "w") as f:
        f.write("# oracle C_l of batch models %s (256 seeded draws, master grid 8000 log-k on "
                "[1e-4,1.0], 3000 tau); columns: model l TT EE TE PP\n" % (C4_MODELS,))
        f.write("# written by tests/golden/make_golden.py with %d oracle threads in %.0f s\n"
                % (oracle.num_threads(), time.time() - t))
        f.writelines(lines)
    print("wrote", out, len(lines), "rows")


def main(name="C2"):
    if name == "C4":
        return main_c4()
    out = os.path.join(HERE, "%s_cl_oracle.txt" % name.lower())
    w = inputs.config(name)
    t = time.time()
    d = oracle.project(w.lmin, w.lmax, w.k, w.tau, w.tau0, w.w_tau, w.S)
    c = oracle.cl(d, w.w_lnk, w.Pk, w.pairs)
    ls = sampled_ells(w.lmin, w.lmax)
    with open(out, "w") as f:
        f.write("# oracle C_l, workload %s (%s); columns: l %s\n"
                % (name, inputs.DESCRIPTIONS[name], " ".join(w.pair_names)))
        f.write("# written by tests/golden/make_golden.py with %d oracle threads in %.0f s\n"
                % (oracle.num_threads(), time.time() - t))
        for l in ls:
            f.write("%d %s\n" % (l, " ".join(repr(float(v)) for v in c[:, l - w.lmin])))
    print("wrote", out, len(ls), "rows")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "C2")
