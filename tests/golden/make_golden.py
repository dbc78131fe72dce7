"""Write oracle reference values for the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``microstructure/``).  Usage:

    python tests/golden/make_golden.py [--jobs J] single_sphere16 spheres64 ...

Each case writes ``tests/golden/oracle_<case>.json`` with the effective
stiffness (six unit Mandel loads), the oracle's iteration counts, the sizes of
the discretisation and the settings used.

With ``--jobs J`` > 1 the discretisation is built once and the six loads are
solved by J forked worker processes that share it copy-on-write (one load per
task, one BLAS thread each).  Every load runs the same oracle solve as in the
serial run; only the loads run side by side.
"""

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import microstructure as ms  # noqa: E402
from oracle.xfem import Discretization  # noqa: E402
from oracle.homogenize import effective_stiffness, solve_loads  # noqa: E402
from oracle.system import System  # noqa: E402

CASES = {
    "single_sphere16": lambda: ms.config_single_sphere(),
    "spheres64": lambda: ms.config_spheres64(),
    "spheres128": lambda: ms.config_spheres128(),
}

_DISC = None      # shared with forked workers


def _solve_one(args):
    k, tol, maxit = args
    t0 = time.perf_counter()
    load = np.eye(6)[k]
    U, infos = solve_loads(_DISC, load[None], tol=tol, maxit=maxit)
    sig = System(_DISC).average_stress(U[0], load)
    print(f"  load {k}: {infos[0]['iters']} iterations, {time.perf_counter() - t0:.0f} s", flush=True)
    return k, sig, int(infos[0]["iters"])


def run(case, tol=1e-13, jobs=1, maxit=20000):
    global _DISC
    cfg = CASES[case]()
    t0 = time.perf_counter()
    disc = Discretization(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], keep_qp=False)
    t1 = time.perf_counter()
    print(case, "setup %.1fs" % (t1 - t0), disc.stats(), flush=True)
    if jobs <= 1:
        C, _, infos = effective_stiffness(disc, tol=tol, maxit=maxit)
        iters = [int(i["iters"]) for i in infos]
    else:
        _DISC = disc
        C = np.zeros((6, 6))
        iters = [0] * 6
        with mp.get_context("fork").Pool(jobs) as pool:
            for k, sig, it in pool.imap_unordered(_solve_one, [(k, tol, maxit) for k in range(6)]):
                C[:, k] = sig
                iters[k] = it
        _DISC = None
    t2 = time.perf_counter()
    out = dict(case=case, n=list(cfg["n"]), tol=tol, c_eff=C.tolist(), iters=iters,
               stats=disc.stats(), seconds_setup=t1 - t0, seconds_solve=t2 - t1, jobs=jobs,
               info={k: v for k, v in cfg["info"].items() if k in ("kind", "vf", "radius")},
               generator="microstructure." + case)
    path = os.path.join(HERE, f"oracle_{case}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(case, "setup %.1fs solve %.1fs" % (t1 - t0, t2 - t1), out["iters"], flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    jobs = 1
    if args and args[0] == "--jobs":
        jobs = int(args[1])
        args = args[2:]
    for c in args:
        run(c, jobs=jobs)
