"""Write oracle_comparator_counts.json: the oracle's per-step iteration
counts of the circulant-preconditioned CG comparators (T. Chan's and
Strang's circulants) of the symmetric Tables 1 and 3 (Section 4) at the grid
sizes the oracle's own tests do not run (2D n + 1 = 128, 256, 512; 3D
n + 1 = 32, 64), with the replication settings (Examples 4.1 / 4.2, x0 = 0,
tol 1e-9, T = 1, M steps as printed).  Calls only oracle/.

    python tests/golden/make_oracle_comparator_counts.py [--workers 6]

Takes about half an hour on 6 cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_comparator_counts.json")


def rows():
    src = json.load(open(os.path.join(HERE, "paper_comparator_iterations.json")))["rows"]
    out = []
    for tab, dim, orders, M, n1, none, tchan, strang in src:
        if tab not in (1, 3):
            continue
        if (dim == 2 and n1 <= 64) or (dim == 3 and n1 <= 16):
            continue
        for kind, it in (("tchan", tchan), ("strang", strang)):
            if it is not None:
                out.append((tab, dim, tuple(orders), M, n1, kind))
    return out


def run_row(row):
    from oracle import cn, examples as ex, operators as op
    tab, dim, orders, M, n1, kind = row
    kp, km = [5.0] * dim, [5.0] * dim          # symmetric tables
    prob = op.Problem(dim, [n1 - 1] * dim, list(orders), kp, km, T=1.0, M=M)
    h = prob.h
    if dim == 2:
        F = lambda m: ex.cell_average(lambda X, Y: ex.ex41_source(
            X, Y, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 0.0), prob.n, h)
    else:
        F = lambda m: ex.cell_average(lambda X, Y, Z: ex.ex42_source(
            X, Y, Z, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y, Z: ex.ex42_exact(X, Y, Z, 0.0), prob.n, h)
    t0 = time.time()
    _, its = cn.run(prob, u0, F, tol=1e-9, x0_mode="zero", maxit=(n1 - 1) ** 3, restart=20,
                    precond=kind)
    return row, [int(v) for v in its], time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    a = ap.parse_args(argv)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    todo = sorted(rows(), key=lambda r: -(r[4] ** r[1]))   # largest first
    res = {}
    with ProcessPoolExecutor(a.workers) as ex:
        for row, its, sec in ex.map(run_row, todo):
            key = f"T{row[0]}-{row[1]}d-{'_'.join(map(str, row[2]))}-{row[4]}-{row[5]}"
            res[key] = {"table": row[0], "dim": row[1], "orders": list(row[2]), "M": row[3],
                        "n_plus_1": row[4], "kind": row[5], "iters": its}
            print(f"{key}: total {sum(its)} ({sec:.0f} s)", flush=True)
    doc = {"source": "oracle/ (cn.run with the circulant comparators, float64), written by "
                     "tests/golden/make_oracle_comparator_counts.py; settings of Section 4's "
                     "replication: Examples 4.1 / 4.2 with k+- = 5, x0 = 0, tol 1e-9, T = 1",
           "rows": dict(sorted(res.items()))}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}: {len(res)} rows")


if __name__ == "__main__":
    main()
