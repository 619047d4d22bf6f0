"""Writes batch4096_switching.json: FP64 oracle results for 64 designs of the batched-island workload.

The designs are rows of the 4096-design batch (inputs.sample_designs(4096, seed=2)), picked to
span the node counts (every 64th row in size order, the largest included), each meshed with its
row index as seed exactly as the batch is.  For each, the oracle integrates the LLG equation with
adaptive Dormand-Prince 5(4) (FP64, rtol = atol = 1e-6) from m = +z to 0.3 ns and records the
switched flag, the switching time and field and the final hard-layer <m_z>.  Only the oracle and
the seeded input generator are used.

Usage: python tests/golden/make_batch_switching.py [threads]
"""
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1603_09493_amd import inputs as I       # noqa: E402

T_END = 0.3e-9
N_DESIGNS = 4096


def pick_rows():
    import numpy as np
    X = I.sample_designs(N_DESIGNS, seed=2)
    n = np.array([I.design_node_target(x) for x in X])
    order = np.argsort(n, kind="stable")
    sel = list(order[::64][:63]) + [int(order[-1])]
    return X, sorted(set(int(q) for q in sel))


def run_one(X, q):
    mesh, mat, fld = I.design_inputs(X[q], seed=q)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    t0 = time.time()
    _, res, _ = om.run(S, [mat], [fld], dict(t_end=T_END, rtol=1e-6))
    r = res[0]
    return dict(row=q, n=mesh.n, switched=int(r["switched"]), t_sw=r["t_sw"], B_sw=r["B_sw"],
                mz_hard=r["mz_hard"], status=r["status"], n_accept=r["n_accept"], n_reject=r["n_reject"],
                seconds=time.time() - t0)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    X, rows = pick_rows()
    rows = sorted(rows, key=lambda q: -I.design_node_target(X[q]))   # largest first
    out = []
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for r in ex.map(lambda q: run_one(X, q), rows):
            out.append(r)
            print(f"row {r['row']} n {r['n']} switched {r['switched']} t_sw {r['t_sw']} {r['seconds']:.0f} s",
                  flush=True)
    out.sort(key=lambda r: r["row"])
    for r in out:
        for k in ("t_sw", "B_sw"):
            if r[k] != r[k]:
                r[k] = None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch4096_switching.json")
    with open(path, "w") as f:
        json.dump({"t_end": T_END, "rtol": 1e-6, "designs": out,
                   "source": "tests/golden/make_batch_switching.py (FP64 oracle)"}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
