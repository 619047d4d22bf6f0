"""Writes parity_floor.txt: how far two FP64 oracle runs of the single-island workload drift apart
when one starts from m0 perturbed by 1e-15 (one unit in the last place of |m|), over the window of
the GPU fixed-step parity test (Dormand-Prince 5 at 10 fs for 0.3 ns).  A GPU-vs-oracle bar of
1e-9 over that window is meaningful only if this floor is far below it.  Uses only the oracle and
the seeded input generator.

Usage: python tests/golden/measure_parity_floor.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1603_09493_amd import inputs as I       # noqa: E402


def main():
    mesh, mat, fld = I.single_island_workload()
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    T, dt = 0.3e-9, 10e-15
    m0 = np.zeros((3, mesh.n))
    m0[2] = 1.0
    rng = np.random.default_rng(11)
    m0p = m0 + 1e-15 * rng.standard_normal(m0.shape)
    rows = []
    for t_end in (0.05e-9, 0.1e-9, 0.2e-9, T):
        opts = dict(t_end=t_end, integrator=O.DP5_FIXED, dt_fixed=dt)
        a, ra, _ = om.run(S, [mat], [fld], opts, m0=m0)
        b, rb, _ = om.run(S, [mat], [fld], opts, m0=m0p)
        rows.append((t_end, float(np.abs(a - b).max()), ra[0]["mz_hard"], ra[0]["switched"]))
        print(rows[-1], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "parity_floor.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle vs itself from m0 + 1e-15 N(0,1) (seed 11), single-island workload\n")
        f.write(f"# ({mesh.n} nodes, 1.2 T at 30 deg ramped in 0.1 ns, alpha 0.1), DP5 fixed dt = 10 fs\n")
        f.write("# written by tests/golden/measure_parity_floor.py\n")
        f.write("# t_end_s  max_abs_dm  mz_hard_at_t_end  switched\n")
        for r in rows:
            f.write(f"{r[0]:.3e} {r[1]:.3e} {r[2]:.6f} {int(r[3])}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
