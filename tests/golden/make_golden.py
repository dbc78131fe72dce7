"""Write oracle reference values for the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``microstructure/``).  Usage:

    python tests/golden/make_golden.py single_sphere16 spheres64 ...

Each case writes ``tests/golden/oracle_<case>.json`` with the effective
stiffness (six unit Mandel loads), the oracle's iteration counts, the sizes of
the discretisation and the settings used.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import microstructure as ms  # noqa: E402
from oracle.xfem import Discretization  # noqa: E402
from oracle.homogenize import effective_stiffness  # noqa: E402

CASES = {
    "single_sphere16": lambda: ms.config_single_sphere(),
    "spheres64": lambda: ms.config_spheres64(),
    "spheres128": lambda: ms.config_spheres128(),
}


def run(case, tol=1e-13):
    cfg = CASES[case]()
    t0 = time.perf_counter()
    disc = Discretization(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], keep_qp=False)
    t1 = time.perf_counter()
    C, U, infos = effective_stiffness(disc, tol=tol, maxit=20000)
    t2 = time.perf_counter()
    out = dict(case=case, n=list(cfg["n"]), tol=tol, c_eff=C.tolist(), iters=[int(i["iters"]) for i in infos],
               stats=disc.stats(), seconds_setup=t1 - t0, seconds_solve=t2 - t1,
               info={k: v for k, v in cfg["info"].items() if k in ("kind", "vf", "radius")},
               generator="microstructure." + case)
    path = os.path.join(HERE, f"oracle_{case}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(case, "setup %.1fs solve %.1fs" % (t1 - t0, t2 - t1), out["iters"], flush=True)


if __name__ == "__main__":
    for c in sys.argv[1:]:
        run(c)
