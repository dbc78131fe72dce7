"""Benchmark: PCG solves per second for the six unit load cases of a 128^3 cell.

Workload (synthetic, seeded): 128^3 voxels, 40 periodic spheres with radii
uniform in [0.06, 0.1] L placed by random sequential addition with a 2-voxel
gap, contrast 10 (E = 10, nu = 0.25 in an E = 1, nu = 0.3 matrix).  One step
solves the six unit Mandel macro strains to the relative tolerance 1e-10 of
the stopping criterion:

* headline (``value``): mixed precision -- FP32 CG inside FP64 iterative
  refinement, the six loads batched in one launch sequence;
* beside it: plain FP64 CG, one load at a time.

Both C_eff are compared with a reference (the oracle's C_eff when its stored
value exists, else an FP64 GPU solve at 1e-13) and their errors are printed.
For the comparison at equal C_eff error, both paths are also run at the
tolerances 1e-8 ... 1e-12 (one timed step each, ``rtol_sweep``).
Setup (level-set classification, enriched numbering, D0, FFT tables) is timed
separately and is not part of a step.

Prints ONE JSON line.  ``--gpus`` above 1 is not supported (single-GPU build).
"""

import argparse
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue rate without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz,
# one add, multiply or fused multiply-add per lane and cycle (FP32 and FP64 alike)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# arithmetic operations per voxel of the regular-voxel operator (six Kuhn tets by
# their 12 shared edges): 36 edge differences, 6 x 12 per tet (3 shear sums,
# trace, 3 normal and 3 shear stresses), 18 edge-force accumulations (the 9
# first-edge and 9 last-edge values each collect two tets; the middle edges one),
# 48 for the corner forces from the edge forces, 24 for the node sums and the
# sign, 3 for lambda V, mu V and 2 mu V
REGULAR_OPS_PER_VOXEL = 36 + 6 * 12 + 18 + 48 + 24 + 3
# copy-like calibration kernel for the HBM byte counters: elementwise negation of
# a float32 buffer reads and writes exactly COPY_BYTES each
COPY_BYTES = 256 << 20
# the end-of-window marker: a negation of this many floats after the timed steps
MARK_ELEMS = 1 << 16
# kernel classes -> substrings of the HIP kernel names
KERNEL_NAMES = {
    "regular_voxels": [r"k_regular<"],
    "irregular_voxels": [r"k_irregular<"],
    "enriched_gather": [r"k_enriched<"],
    "fft_x_forward": [r"k_fft_plane_fwd<", r"k_fft_x_fwd(_t)?<"],
    "fft_y_forward": [r"k_fft_y(_t)?<{t}(, \d+, \d+)?, false>"],
    "fft_z_green": [r"k_fft_z_t<", r"k_fft_z_green<"],
    "fft_y_inverse": [r"k_fft_y(_t)?<{t}(, \d+, \d+)?, true>"],
    "fft_x_inverse": [r"k_fft_plane_inv<", r"k_fft_x_inv(_t)?<"],
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(g, s, nrhs):
    """Algorithmic HBM bytes per launch of each kernel class (one CG iteration)
    processing nrhs loads (may be fractional: the mean over launches).

    g: dict with N, nX, nirr, n0, n1, n2; s: bytes per real (4 or 8).  The
    regular-voxel operator moves 2F per load (read d, write z) plus one byte of
    material per voxel once per launch, and the launch also carries the
    enriched gather.
    """
    N, nX, nirr = g["N"], g["nX"], g["n_irregular_voxels"]
    nh = g["n0"] // 2 + 1
    specN = g["n2"] * g["n1"] * nh               # complex entries per component
    spec = 3 * specN * 2 * s                     # one 3-component half spectrum
    field = 3 * N * s                            # one 3-component nodal field
    gather = nX * (8 * 4 + 3 * s)                # enriched gather: source ids, write z~
    per = {
        # read d, write z; the launch also runs the enriched gather (material: below)
        "regular_voxels": 2 * field + gather,
        # u, level set, enriched ids, labels, scaled enriched d, corner forces; moments per cut element
        "irregular_voxels": nirr * (8 * 3 * s + 8 * s + 8 * 4 + 12 * 4 + 8 * 3 * s + 48 * s)
                            + g.get("n_cut_elements", 0) * 12 * s,
        "enriched_gather": gather,
        "fft_x_forward": 3 * field + spec,                        # read f, z; write f, spectrum
        "fft_y_forward": 2 * spec,
        "fft_z_green": 2 * spec + nX * 3 * s * 3,                 # + enriched residual update
        "fft_y_inverse": 2 * spec,
        "fft_x_inverse": spec + 4 * field + nX * 3 * s * 5,       # read spectrum, d, u; write d, u; + enriched
        "enriched_residual": nX * 3 * s * 3,
        "enriched_update": nX * 3 * s * 5,
        "scalars": 0,
    }
    out = {k: v * nrhs for k, v in per.items()}
    out["regular_voxels"] += N                   # one byte of material per voxel, once per launch
    return out


def source_digest():
    """SHA-256 over the HIP sources and the C header (the counters belong to this code)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_02172_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "xfft.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _kernel_class(name):
    prec = "fp32" if "<float" in name else "fp64" if "<double" in name else None
    if prec is None:
        return None
    t = "float" if prec == "fp32" else "double"
    for k, pats in KERNEL_NAMES.items():
        if any(re.search(p.replace("{t}", t), name) for p in pats):
            return k, prec
    return None


def pmc_summary(fetch_csv, write_csv):
    """Mean HBM bytes per dispatch of every kernel class from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, both in KiB), scaled by the counter readings of the
    calibration copy (reads and writes COPY_BYTES).  Only the dispatches of the timed
    steps count: those between the calibration copy and the end marker."""
    import csv
    per = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                key = int(row["Dispatch_Id"])
                rows.setdefault(key, [row["Kernel_Name"], 0.0])[1] += float(row["Counter_Value"]) * 1024.0
        negs = sorted(k for k, (n, v) in rows.items() if "neg_kernel" in n)
        if len(negs) < 2:
            raise SystemExit(f"no calibration copy and end marker in {path}")
        first, last = negs[0], negs[-1]
        factor = COPY_BYTES / rows[first][1]
        per[counter] = factor
        for k, (n, v) in rows.items():
            if not first < k < last:
                continue
            kc = _kernel_class(n)
            if kc is None:
                continue
            d = per.setdefault(f"{kc[0]}/{kc[1]}", {})
            d.setdefault(counter, []).append(v)
    out = {"source_sha256": source_digest(), "copy_bytes": COPY_BYTES,
           "factor_fetch": per.pop("FETCH_SIZE"), "factor_write": per.pop("WRITE_SIZE"), "kernels": {}}
    for k, d in sorted(per.items()):
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            fb = float(np.mean(d["FETCH_SIZE"])) * out["factor_fetch"]
            wb = float(np.mean(d["WRITE_SIZE"])) * out["factor_write"]
            out["kernels"][k] = {"dispatches": len(d["FETCH_SIZE"]), "fetch_bytes": round(fb),
                                 "write_bytes": round(wb), "bytes_per_launch": round(fb + wb)}
    return out


def load_traffic(workload):
    """Calibrated HBM bytes per launch from the committed counter summary, if it
    was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    a = text.find("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    data = json.loads(text[a + 7:b])
    if data.get("source_sha256") != source_digest():
        log("counter summary was taken on other sources: traffic null")
        return None
    return data


def cpu_model():
    """Model name of the host CPU (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg, fp64_iters, sample_cut=8000, sample_iters=2):
    """Time the CPU oracle on a bounded sample of the workload and scale to solves/s.

    The oracle runs single-threaded (BLAS and FFT thread pools limited to one
    thread); ``cores`` is that thread count, and the host's CPU model and
    logical CPU count are reported beside it."""
    from threadpoolctl import threadpool_limits
    from oracle.xfem import Discretization
    from oracle.system import System
    from oracle.green import GreenOperator
    from oracle.solver import pcg
    with threadpool_limits(1):
        d = Discretization(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], keep_qp=False,
                           sample_cut=sample_cut)
        ncut = len(d.cut_voxel)
        t_setup = d.timing["uncut"] + d.timing["cut"] * ncut / max(d.timing["cut_built"], 1)
        # assembly of the system and the Green operator (part of the oracle's work)
        t0 = time.perf_counter()
        s = System(d)
        g = GreenOperator(d.n)
        eb = np.eye(6)[0]
        b = s.rhs(eb)
        t_sys = time.perf_counter() - t0
        t0 = time.perf_counter()
        pcg(s.apply, b, lambda f: g.apply(f, d.nX), lambda x: s.average_stress(x, eb), d.volume, 0.0,
            sample_iters)
        t_iter = (time.perf_counter() - t0) / sample_iters
    total = t_setup + t_sys + float(np.sum(fp64_iters)) * t_iter
    return dict(value=6.0 / total, unit="solves/s", cores=1, kind="oracle",
                cpu_model=cpu_model(), host_logical_cpus=os.cpu_count(),
                sample=(f"oracle setup with {min(sample_cut, ncut)} of {ncut} cut elements built "
                        f"(scaled to all), system assembly, {sample_iters} PCG iterations of one load at full "
                        f"size; scaled to 6 loads x the FP64 path's iteration counts ({int(np.sum(fp64_iters))} "
                        f"total); 1 thread"),
                seconds_setup_est=t_setup, seconds_assembly=t_sys, seconds_per_iteration=t_iter)


def extrapolation_check(rtol, sample_cut=40, sample_iters=2):
    """The cpu_baseline extrapolation checked where the oracle also runs in full:
    the 16^3 single-sphere cell, one load.  Returns the extrapolated and the
    measured seconds (setup plus solve to rtol, one thread)."""
    from threadpoolctl import threadpool_limits
    import microstructure as ms
    from oracle.xfem import Discretization
    from oracle.system import System
    from oracle.green import GreenOperator
    from oracle.solver import pcg
    cfg = ms.config_single_sphere()
    eb = cfg["loads"][0]
    with threadpool_limits(1):
        # full run: setup with every cut element built, PCG to the tolerance
        t0 = time.perf_counter()
        d = Discretization(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], keep_qp=False)
        s = System(d)
        g = GreenOperator(d.n)
        b = s.rhs(eb)
        _, info = pcg(s.apply, b, lambda f: g.apply(f, d.nX), lambda x: s.average_stress(x, eb), d.volume,
                      rtol, 100000)
        t_full = time.perf_counter() - t0
        # the same extrapolation as the baseline: sampled setup, a few timed iterations
        ds = Discretization(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], keep_qp=False,
                            sample_cut=sample_cut)
        t_setup = ds.timing["uncut"] + ds.timing["cut"] * len(ds.cut_voxel) / max(ds.timing["cut_built"], 1)
        t0 = time.perf_counter()
        s2, g2 = System(ds), GreenOperator(ds.n)
        b2 = s2.rhs(eb)
        t_sys = time.perf_counter() - t0
        t0 = time.perf_counter()
        pcg(s2.apply, b2, lambda f: g2.apply(f, ds.nX), lambda x: s2.average_stress(x, eb), ds.volume, 0.0,
            sample_iters)
        t_iter = (time.perf_counter() - t0) / sample_iters
    t_est = t_setup + t_sys + int(info["iters"]) * t_iter
    return dict(workload="single_sphere16, 1 load, rtol %g" % rtol, iters=int(info["iters"]),
                seconds_measured=round(t_full, 3), seconds_extrapolated=round(t_est, 3),
                ratio=round(t_est / t_full, 3))


def bench_uneven(args):
    """Sixteen RVEs of uneven size (32..128)^3, six loads each: 96 solves as one
    captured graph (mixed precision), against the same problems solved one
    after the other, and C_eff against FP64 solves at rtol 1e-13."""
    import torch
    import microstructure as ms
    from paper_2601_02172_amd import Problem, batch_effective_stiffness
    t0 = time.perf_counter()
    cfgs = ms.config_uneven_batch()
    log(f"16 RVEs generated in {time.perf_counter() - t0:.1f}s: n = {[c['n'][0] for c in cfgs]}")
    probs = [Problem(c["n"], c["length"], c["L"], c["phase"], c["lame"], rtol=args.rtol, precision="mixed",
                     inner_rtol=args.inner_rtol) for c in cfgs]
    try:
        for _ in range(args.warmup):
            batch_effective_stiffness(probs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Cb, st = batch_effective_stiffness(probs, with_stats=True)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / args.steps
        # the same problems one after the other (each with its six loads batched)
        for p in probs:
            p.effective_stiffness()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for p in probs:
                p.effective_stiffness()
        torch.cuda.synchronize()
        t_seq = (time.perf_counter() - t0) / args.steps
    finally:
        for p in probs:
            p.close()
    errs = []
    for i, c in enumerate(cfgs):
        with Problem(c["n"], c["length"], c["L"], c["phase"], c["lame"], rtol=1e-13) as pr:
            C_ref = pr.effective_stiffness()[0]
        errs.append(float(np.linalg.norm(Cb[i] - C_ref) / np.linalg.norm(C_ref)))
    nsolve = 6 * len(cfgs)
    log(f"batch: {1000 * t_batch:.1f} ms for {nsolve} solves; one RVE after the other: {1000 * t_seq:.1f} ms; "
        f"max C_eff rel error {max(errs):.2e}")
    out = {
        "metric": "PCG solves/sec, 16 uneven RVEs x 6 loads as one batch (mixed)",
        "value": round(nsolve / t_batch, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000 * t_batch, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP64 refinement)", "data": "synthetic",
        "config": {"workload": "uneven16: 16 RVEs n in {32,48,64,96,128}, spheres vf 0.1-0.3 (achieved "
                   f"{min(c['info']['vf'] for c in cfgs):.2f}-{max(c['info']['vf'] for c in cfgs):.2f}), contrast 100",
                   "rtol": args.rtol, "inner_rtol": args.inner_rtol, "voxels": int(sum(np.prod(c["n"]) for c in cfgs))},
        "roofline": None, "cpu_baseline": None,
        "sequential_solves_per_s": round(nsolve / t_seq, 4),
        "c_eff_rel_error_max": max(errs), "iters": np.asarray(st["iters"]).tolist(),
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--inner-rtol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the tolerance sweep (C_eff error and time of both paths at rtol 1e-8 ... 1e-12)")
    ap.add_argument("--schemes", action="store_true",
                    help="also time the FP64 solution schemes (linear CG, nonlinear CG, Barzilai-Borwein, basic), "
                         "6 loads batched, one step each")
    ap.add_argument("--workload", default="spheres128", choices=["spheres128", "ellipsoids256", "uneven16"])
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs of this script (FETCH_SIZE, WRITE_SIZE) as JSON")
    args = ap.parse_args()
    if args.pmc_summary:
        print(json.dumps(pmc_summary(*args.pmc_summary), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(load cases and RVEs would be sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import microstructure as ms
    from paper_2601_02172_amd import Problem

    torch.cuda.init()
    if args.workload == "uneven16":
        return bench_uneven(args)
    t_gen = time.perf_counter()
    if args.workload == "spheres128":
        cfg = ms.config_spheres128()
        wl_desc = "spheres128: 128^3, 40 RSA spheres r~U[0.06,0.1]L, contrast 10, 6 unit loads"
    else:
        log("generating the 256^3 ellipsoid microstructure (about a minute on the host)")
        cfg = ms.config_ellipsoids()
        wl_desc = ("ellipsoids256: 256^3, 200 random prolate spheroids (aspect 3), vf 0.20, "
                   "per-inclusion lognormal Lame pairs, 6 unit loads")
    log(f"inputs ready in {time.perf_counter() - t_gen:.1f}s")
    E = np.eye(6)

    def make(precision, batch):
        return Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=args.rtol,
                       precision=precision, batch=batch, inner_rtol=args.inner_rtol)

    t0 = time.perf_counter()
    pm = make("mixed", True)
    setup_s = time.perf_counter() - t0
    lay = pm.layout(with_arrays=False)
    lay.update(n0=cfg["n"][0], n1=cfg["n"][1], n2=cfg["n"][2])
    log(f"setup {setup_s:.3f}s, nX={lay['nX']}, irregular voxels={lay['n_irregular_voxels']}")

    for _ in range(args.warmup):
        pm.solve(E, c_eff=True)
    torch.cuda.synchronize()
    # calibration copy for the byte counters, right before the timed steps; a
    # small negation after them marks the end of the counted window
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.neg(src)
    mark = torch.ones(MARK_ELEMS, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    del src, dst
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r_mixed = pm.solve(E, c_eff=True)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    torch.neg(mark)
    torch.cuda.synchronize()
    # the same steps again with a HIP event before and after every kernel launch
    # (launched one by one instead of by graph replay; kernel durations are the same)
    pm.profile_begin()
    for _ in range(args.steps):
        pm.solve(E, c_eff=True)
    region = pm.profile_end()
    ms_per_step = 1000.0 * t_mixed / args.steps
    value = 6.0 * args.steps / t_mixed
    log(f"mixed: {ms_per_step:.1f} ms/step, inner iters {list(r_mixed['iters'])}, outer {list(r_mixed['outer_iters'])}")

    fp64 = None
    if not args.no_fp64:
        p64 = make("fp64", False)
        p64.solve(E[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r64 = p64.solve(E, c_eff=True)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        fp64 = dict(value=6.0 * args.steps / t64, ms_per_step=1000.0 * t64 / args.steps,
                    iters=[int(v) for v in r64["iters"]])
        log(f"fp64 plain: {fp64['ms_per_step']:.1f} ms/step, iters {fp64['iters']}")

    schemes = None
    if args.schemes:
        schemes = {}
        for name in ("lcg", "nlcg", "bb", "basic"):
            ps = Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=args.rtol,
                         precision="fp64", scheme=name, maxit=20000)
            ps.solve(E[:1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = ps.solve(E, c_eff=True)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            ps.close()
            schemes[name] = dict(ms_per_step=round(1000.0 * ts, 3), solves_per_s=round(6.0 / ts, 4),
                                 iters=[int(v) for v in rs["iters"]], converged=bool(rs["converged"]),
                                 c_eff=rs["c_eff"])
            log(f"scheme {name} (fp64, 6 loads batched): {1000.0 * ts:.1f} ms, iters {schemes[name]['iters']}")

    # accuracy of both paths against a reference C_eff
    golden = os.path.join(ROOT, "tests", "golden", f"oracle_{args.workload}.json")
    if os.path.exists(golden):
        C_ref = np.array(json.load(open(golden))["c_eff"])
        ref_kind = "oracle"
    else:
        pref = Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=1e-13)
        C_ref = pref.effective_stiffness()[0]
        pref.close()
        ref_kind = "gpu_fp64_rtol1e-13"
    nrm = np.linalg.norm(C_ref)
    err_mixed = float(np.linalg.norm(r_mixed["c_eff"] - C_ref) / nrm)
    err_fp64 = float(np.linalg.norm(r64["c_eff"] - C_ref) / nrm) if fp64 else None

    log(f"C_eff rel error vs {ref_kind}: mixed {err_mixed:.2e}, fp64 {err_fp64}")
    if schemes:
        for v in schemes.values():
            v["c_eff_rel_error"] = float(np.linalg.norm(v.pop("c_eff") - C_ref) / nrm)
    # equal-error comparison: both paths over a range of tolerances, one timed
    # step each after one untimed solve (autotuning, graph capture)
    sweep = None
    if not args.no_sweep and fp64 and args.workload == "spheres128":
        sweep = []
        for rt in (1e-8, 1e-9, 1e-10, 1e-11, 1e-12):
            row = {"rtol": rt}
            for name, prec, batch in (("mixed", "mixed", True), ("fp64", "fp64", False)):
                q = Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=rt,
                            precision=prec, batch=batch, inner_rtol=args.inner_rtol)
                q.solve(E, c_eff=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rq = q.solve(E, c_eff=True)
                torch.cuda.synchronize()
                tq = time.perf_counter() - t0
                q.close()
                row[name] = dict(ms_per_step=round(1000.0 * tq, 3), solves_per_s=round(6.0 / tq, 3),
                                 c_eff_rel_error=float(np.linalg.norm(rq["c_eff"] - C_ref) / nrm))
            log(f"rtol {rt:g}: mixed {row['mixed']['ms_per_step']} ms err {row['mixed']['c_eff_rel_error']:.2e}; "
                f"fp64 {row['fp64']['ms_per_step']} ms err {row['fp64']['c_eff_rel_error']:.2e}")
            sweep.append(row)
    # dominant kernel of the timed region: largest total time among all launches
    byts = {"fp32": algorithmic_bytes(lay, 4, 6), "fp64": algorithmic_bytes(lay, 8, 6)}
    totals = {k: m * c for k, (m, c) in region.items()}
    dom_key = max(totals, key=totals.get)
    dom, dom_prec = dom_key
    dom_ms, dom_n = region[dom_key]
    # bytes per launch: the timed region mixes launches with 6..1 active loads; scale
    # the 6-load figure by the mean number of active loads per launch
    # CG-loop launches skip loads that have converged: the mean number of loads a
    # launch processes is (load-iterations in the timed steps) / (launches)
    if dom_prec == "fp32":
        active = min(6.0, float(np.sum(r_mixed["iters"])) * args.steps / max(dom_n, 1))
    else:
        active = 6.0
    bytes_launch = algorithmic_bytes(lay, 4 if dom_prec == "fp32" else 8, active)[dom]
    achieved = bytes_launch / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    traffic = None
    tr = load_traffic(args.workload)
    if tr is not None and f"{dom}/{dom_prec}" in tr["kernels"]:
        traffic = tr["kernels"][f"{dom}/{dom_prec}"]["bytes_per_launch"]
    # The path streams nodal fields (no dense contraction), so the roof reported is
    # HBM bandwidth: algorithmic bytes per launch over the launch time against
    # 8 TB/s.  For the regular-voxel operator, whose arithmetic per voxel is fixed
    # by the edge form, the VALU issue fraction is reported beside it.
    ops_launch = REGULAR_OPS_PER_VOXEL * lay["N"] * active if dom == "regular_voxels" else None
    valu = None
    if ops_launch:
        tops = ops_launch / (dom_ms * 1e-3) / 1e12
        valu = dict(achieved=round(tops, 3), peak=round(VALU_PEAK_TOPS, 2),
                    unit="Tops/s (VALU lane operations, no packed FP32)", frac=round(tops / VALU_PEAK_TOPS, 4),
                    ops_per_launch=int(ops_launch), ops_per_voxel=REGULAR_OPS_PER_VOXEL)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=f"{dom} ({dom_prec})", bytes_per_launch=int(bytes_launch),
                    ms_per_launch=round(dom_ms, 5), launches=dom_n, mean_active_loads=round(active, 3),
                    traffic_over_algorithmic=round(traffic / bytes_launch, 3) if traffic else None,
                    valu=valu)
    # per-kernel breakdown of one CG iteration with all six loads active
    prof = pm.profile(precision="fp32", nrhs=6, nrep=10)
    kernels = {k: dict(ms=round(v[0], 5), launches_per_iter=v[1] / 10.0,
                       gbs=round(byts["fp32"][k] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 and byts["fp32"][k] else None)
               for k, v in prof.items()}
    region_summary = {f"{k[0]}/{k[1]}": [round(v[0], 5), v[1]] for k, v in region.items() if v[1]}
    log(f"dominant kernel {dom}: {dom_ms:.4f} ms, {achieved:.0f} GB/s, roofline {roofline['bound']} "
        f"frac {roofline['frac']}")
    grad_info = None
    if args.workload == "ellipsoids256":
        # loss ||C_eff - C_t||_F^2 with C_t = C_eff at the median moduli; gradient over all Lame pairs
        lame_med = cfg["lame"].copy()
        lame_med[1:] = np.median(cfg["lame"][1:], axis=0)
        pm.set_lame(lame_med)
        C_t = pm.effective_stiffness()[0]
        pm.set_lame(cfg["lame"])
        C_now = pm.effective_stiffness()[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, _ = pm.grad_lame(2.0 * (C_now - C_t))
        t_grad = time.perf_counter() - t0
        grad_info = dict(parameters=int(g.size), seconds=round(t_grad, 4), loss=float(np.sum((C_now - C_t) ** 2)),
                         grad_norm=float(np.linalg.norm(g)))
        log(f"gradient over {g.size} Lame parameters in {t_grad:.3f}s")
    cpu = None
    if not args.no_cpu_baseline and fp64 and args.workload == "spheres128":
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(cfg, fp64["iters"])
        cpu["extrapolation_check"] = extrapolation_check(args.rtol)
        log(f"cpu baseline {cpu['value']:.3e} solves/s; extrapolation check {cpu['extrapolation_check']}")

    out = {
        "metric": "PCG solves/sec (6 loads, 128^3) mixed vs FP64 plain at equal C_eff error",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 refinement)",
        "data": "synthetic",
        "config": {"workload": wl_desc,
                   "rtol": args.rtol, "inner_rtol": args.inner_rtol, "precision": "mixed", "batched_loads": 6,
                   "n_enriched": lay["nX"], "n_irregular_voxels": lay["n_irregular_voxels"],
                   "vf": cfg["info"]["vf"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_plain": fp64,
        "c_eff_rel_error": {"mixed": err_mixed, "fp64": err_fp64, "reference": ref_kind},
        "inner_iters": [int(v) for v in r_mixed["iters"]],
        "outer_iters": [int(v) for v in r_mixed["outer_iters"]],
        "setup_seconds": round(setup_s, 4),
        "kernels": kernels,
        "timed_region_kernels": region_summary,
        "loss_gradient": grad_info,
        "schemes": schemes,
        "rtol_sweep": sweep,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
