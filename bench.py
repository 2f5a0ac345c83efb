"""Benchmark: requests/s (and request p50/p99 latency) of the whole dense BEM hot path on one MI355X.

Default workload: the serving mix (`meshgen.mixed_stream`, seed 5, Poisson arrivals at 2
requests/s): spheres, 1.0/0.6/0.4 ellipsoids and cubes of 320-20000 triangles, eps_r 1.5-10,
k0 a 0.5-10, 1-64 random plane waves each - seeded synthetic input.  One step = one request:
load the mesh (host topology), assemble every operator on the device (L^A, L^phi, K~ at the
object and background wavenumbers, near corrections, gathers, the nested-solve inverse and the
block preconditioner) and solve the final system for all its plane waves to a 1e-6 relative
float64 residual, the requests admitted by the HBM budget and overlapping on the device.  The
same stream is served in BEM_FP32 (the headline), mixed precision and float64.  `--workload`
selects one problem solved per step instead (c1, c2, c2x256, c3, spharr, c4), and
`--serve-sweep` an arrival-rate sweep of the mix.

Reported beside the throughput:
  roofline      the dominant kernel class of a sequential pass over the timed requests,
                measured with HIP events on its launch stream (library profiler): achieved
                algorithmic TFLOP/s vs the matrix peak for the GEMMs and the Gauss-Jordan
                update, GB/s vs 8 TB/s HBM for the GEMV, with the HBM bytes per launch from
                rocprofv3 counters beside it;
  fill_GBps     bytes of the float64 dense blocks written / device fill time;
  cpu_baseline  the float64 CPU oracle solving whole requests of the stream, smallest first,
                for about 20 s of host time (fills over every host core, augmented system by
                LAPACK LU), as solves/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBPS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP64_MFMA_PEAK_TFLOPS = 78.6   # dense float64 matrix peak (the same figure as the vector one)
FP32_MFMA_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    import meshgen
    return {"c1": meshgen.config_c1, "c2": meshgen.config_c2, "c2x256": meshgen.config_c2_multi,
            "c3": meshgen.config_c3, "spharr": meshgen.config_sphere_array, "c4": meshgen.config_c4}[name]()


def cpu_baseline(w, n_sample: int = 12) -> dict:
    """Oracle timed on a bounded sample: n_sample test triangles of each of the four dense fills
    (L at two wavenumbers, K~ at two), scaled by N_T / n_sample, plus a dense LU of size 2048
    scaled by (N_aug / 2048)^3 to the augmented system the oracle solves."""
    import numpy as np
    import scipy.linalg as sla
    from threadpoolctl import threadpool_info

    from oracle import constants as OC
    from oracle import mesh as OM
    from oracle import operators as OO

    topo = OM.build_topology(w.xyz, w.tri, w.obj)
    bary = OM.buffa_christiansen(topo)
    near = OO.near_pairs(topo)
    bcd = OO.bc_on_subtriangles(bary)
    k0 = OC.k0_of(w.freq_hz)
    k_int = OC.wavenumber(k0, OC.eps_c(w.eps_r[0], w.sigma[0], w.freq_hz), w.mu_r[0])
    k_bg = OC.wavenumber(k0, 1.0, 1.0)
    nt, ne = len(topo.tri), len(topo.edges)
    rng = np.random.default_rng(0)
    subset = np.sort(rng.choice(nt, size=min(n_sample, nt), replace=False))
    t0 = time.perf_counter()
    for k in (k_int, k_bg):
        OO.fill_L(topo, k, near, test_subset=subset)
        OO.fill_K(topo, bary, k, near, bcd, test_subset=subset)
    t_fill = (time.perf_counter() - t0) * nt / len(subset)
    n_lu = 2048
    A = rng.standard_normal((n_lu, n_lu)) + 1j * rng.standard_normal((n_lu, n_lu))
    t0 = time.perf_counter()
    sla.lu_factor(A, overwrite_a=True, check_finite=False)
    t_lu_small = time.perf_counter() - t0
    n_aug = 3 * ne + 2 * (nt - 1)
    t_lu = t_lu_small * (n_aug / n_lu) ** 3
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"value": 1.0 / (t_fill + t_lu), "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(subset)} of {nt} test triangles of the 4 dense fills (x{nt / len(subset):.0f}) "
                      f"+ LU of a {n_lu}^2 complex matrix scaled by (N_aug={n_aug}/{n_lu})^3; "
                      f"fill est {t_fill:.1f} s, LU est {t_lu:.1f} s"}


def kernel_source_digest(regions) -> str | None:
    """sha256 over the code of a kernel: each region is [file, begin, end] (from the first
    occurrence of `begin`, "" for the file start, up to the next `end`); // comments, trailing
    blanks and empty lines are left out, so that only a change of the code itself counts."""
    import hashlib
    h = hashlib.sha256()
    for rel, begin, end in regions:
        path = ROOT / rel
        if not path.exists():
            return None
        text = path.read_text()
        i = text.find(begin)
        j = text.find(end, i) if i >= 0 else -1
        if i < 0 or j < 0:
            return None
        for line in text[i:j].splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update((code + "\n").encode())
    return h.hexdigest()


def measured_traffic(kernel_class: str):
    """HBM bytes per launch of a kernel class from the committed counter summary
    (profiles/traffic.json), or None when the kernel's source (its listed regions) changed
    since it was measured."""
    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    entry = json.loads(path.read_text()).get(kernel_class)
    if not entry or kernel_source_digest(entry["source_regions"]) != entry["source_sha256"]:
        return None
    return float(entry["hbm_bytes_per_launch"])


def copy_calibration() -> int:
    """A plain device copy of known size (256 MiB read + 256 MiB written per dispatch, 5
    dispatches): the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 5 x 256 MiB", flush=True)
    return 0


def _oracle_assemble_parallel(w, procs: int):
    """The oracle's four dense fills split by test triangle over `procs` host processes (rows
    summed in a fixed chunk order), then its Operators record - the same arithmetic as
    oracle.systems.assemble, on every host core."""
    import multiprocessing as mp

    import numpy as np

    from oracle import constants as OC
    from oracle import mesh as OM
    from oracle import operators as OO
    from oracle import systems as OS

    topo = OM.build_topology(w.xyz, w.tri, w.obj)
    bary = OM.buffa_christiansen(topo)
    bcd = OO.bc_on_subtriangles(bary)
    near = OO.near_pairs(topo)
    _ORACLE_SHARED.update(topo=topo, bary=bary, bcd=bcd, near=near)
    nt, ne = len(topo.tri), len(topo.edges)
    k0 = OC.k0_of(w.freq_hz)
    epsc = OC.eps_c(w.eps_r[0], w.sigma[0], w.freq_hz)
    k_int = OC.wavenumber(k0, epsc, w.mu_r[0])
    k_bg = OC.wavenumber(k0, w.eps_bg, w.mu_bg)
    chunks = [list(range(i, nt, 4 * procs)) for i in range(4 * procs)]
    mats = {}
    with mp.get_context("fork").Pool(procs, initializer=_oracle_worker_init) as pool:
        for name, k in (("int", k_int), ("bg", k_bg)):
            LA, Lp, K = np.zeros((ne, ne), complex), np.zeros((nt, nt), complex), np.zeros((ne, ne), complex)
            for er, la, tr, lp, kk in pool.imap(_oracle_rows, [(k, c) for c in chunks]):
                LA[er] += la
                Lp[tr] += lp
                K[er] += kk
            mats[name] = (LA, Lp, K)
    Ix = OO.gram_Ix(topo, bary, bcd)
    D = OM.incidence_D(topo).toarray()
    Bm, F, _ = OM.charge_maps(topo)
    return OS.Operators(topo, bary, D, Bm.toarray(), F.toarray(), Ix, *mats["int"], *mats["bg"], mats["bg"][2], k0,
                        [k_int], k_bg, [epsc], list(w.mu_r), complex(w.eps_bg), float(w.mu_bg))


_ORACLE_SHARED: dict = {}


def _oracle_worker_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _oracle_rows(args):
    import numpy as np

    from oracle import operators as OO
    k, subset = args
    g = _ORACLE_SHARED
    LA, Lp = OO.fill_L(g["topo"], k, g["near"], test_subset=subset)
    K = OO.fill_K(g["topo"], g["bary"], k, g["near"], g["bcd"], test_subset=subset)
    er = np.unique(g["topo"].tri_edges[subset].ravel())
    return er, LA[er], np.asarray(subset), Lp[subset], K[er]


def serve_cpu_baseline(requests, budget_s: float = 20.0) -> dict:
    """The oracle solving whole requests of the stream, smallest first, until `budget_s` of host
    wall time is spent (at least one): fills on every host core, the augmented system (eqs.
    AEFIEintdis, AEFIEeqvdis, AEFIEextdis) by LAPACK LU for all the request's plane waves."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import systems as OS

    procs = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    done, t_total, names = 0, 0.0, []
    for w in sorted(requests, key=lambda w: (len(w.tri), len(w.khat))):
        t0 = time.perf_counter()
        ops = _oracle_assemble_parallel(w, procs)
        b = np.stack([OS.rhs(ops, w.khat[i], w.pol[i]) for i in range(len(w.khat))], axis=1)
        OS.solve_augmented(ops, b)
        t_total += time.perf_counter() - t0
        done += 1
        names.append(f"{w.name} ({len(w.tri)} triangles)")
        if t_total >= budget_s:
            break
    blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / t_total, "unit": "solves/s", "cores": int(procs), "kind": "oracle",
            "sample": f"{done} whole request(s) of the timed stream, smallest first, timed end to end "
                      f"(fill on {procs} processes, augmented LU with {blas} BLAS threads): " + "; ".join(names),
            "seconds": t_total, "host_cpu": cpu, "nproc": os.cpu_count()}


def _dense_bytes(nt: int) -> float:
    """float64 bytes of the dense blocks one single-object request fills: L^A, L^phi at the
    background wavenumber, L^A, L^phi, K~ at the object's, K~ at the background's."""
    ne = 1.5 * nt
    return 16.0 * (4 * ne * ne + 2.0 * nt * nt)


def _serve_once(B, stream, prec, args):
    """Submit the stream's requests at their arrival times on a fresh context, poll until all are
    final.  Returns the per-request records, the wall time from the first arrival to the last
    completion, and the combiner counters."""
    import torch

    ctx = B.bem_create(0)
    opts = B.solve_opts(tol=args.tol, restart=args.restart, maxit=args.maxit, max_refine=8)

    def request(w):
        p = B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, precision=prec)
        return B.Request(w.xyz, w.tri, w.obj, p, B.plane_waves(w.khat, w.pol), opts)

    warm, timed = stream[:args.warmup], stream[args.warmup:]
    # warm-up requests, all at once, untimed (kernel loading, allocator, host threads)
    held = [request(w) for _, w in warm]  # the outputs must outlive the requests
    tickets = [B.bem_submit(ctx, r) for r in held]
    B.bem_drain(ctx)
    for t in tickets:
        try:
            B.bem_poll(ctx, t)
        except B.BemError as e:
            log(f"  warm-up request failed: {e}")
    torch.cuda.synchronize()
    reqs = [(at - timed[0][0], request(w), w) for at, w in timed]
    pending, recs = {}, []
    t0 = time.perf_counter()
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i][0] <= now:
            pending[B.bem_submit(ctx, reqs[i][1])] = reqs[i]
            i += 1
        for tk in list(pending):
            try:
                rc, info = B.bem_poll(ctx, tk)
            except B.BemError as e:
                rc, info = e.code, None
                log(f"  {pending[tk][2].name}: {e}")
            if rc != B.BEM_PENDING:
                _, r, w = pending.pop(tk)
                recs.append({"name": w.name, "nt": len(w.tri), "nexc": len(w.khat), "status": int(rc) if isinstance(rc, int) else -99,
                             "latency": info.seconds if info else float("nan"),
                             "outer": info.outer_iters if info else -1,
                             "res": info.rel_residual if info else float("nan")})
                log(f"  {w.name:36s} status {recs[-1]['status']:3d} latency {recs[-1]['latency']:7.3f} s "
                    f"outer {recs[-1]['outer']:5d} res {recs[-1]['res']:.1e}")
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    comb = B.bem_serve_stats(ctx)
    B.bem_destroy(ctx)
    return recs, wall, comb


def _profiled_pass(B, timed, args, prec):
    """The timed requests once more, one after another (mesh load, assembly in the headline
    precision, solve), with HIP events recorded around every launch on its stream: per-class
    device time, algorithmic bytes and work of each kernel class without the overlap of
    concurrent requests."""
    ctx = B.bem_create(0)
    opts = B.solve_opts(tol=args.tol, restart=args.restart, maxit=args.maxit, max_refine=8)
    B.bem_profile_enable(True)
    for w in timed:
        mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
        info = B.bem_mesh_info(ctx, mesh)
        op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, precision=prec))
        rc, _, _, _, si = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol), opts, info["n_edge"], info["n_tri"])
        B.bem_release(ctx, op)
        B.bem_release(ctx, mesh)
        log(f"  profiled {w.name:36s} status {rc} outer {si.outer_iters}")
    prof = {k: B.bem_profile_read(k) for k in range(len(B.KC_NAMES))}
    B.bem_profile_enable(False)
    B.bem_destroy(ctx)
    return prof


def _class_roofline(B, dom, p) -> dict:
    """Bound, achieved rate (algorithmic bytes or flops over the class's event-timed launch
    time), peak and fraction of one kernel class."""
    if dom in (B.KC_GEMV_F64, B.KC_GEMV_F32, B.KC_GATHER):
        achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS}
    elif dom == B.KC_GEMM_F32:
        achieved = p["work"] / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_MFMA_PEAK_TFLOPS}
    elif dom in (B.KC_DENSE_INV, B.KC_GEMM_F64):
        achieved = p["work"] / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_MFMA_PEAK_TFLOPS}
    else:
        # fill: about 64 float64 vector operations per Green's-function evaluation
        achieved = p["work"] * 64 / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS}
    return roof


def _kernel_classes(B, prof) -> dict:
    """Every timed kernel class of a profiled pass: its time, launches and roofline."""
    out = {}
    for k, p in prof.items():
        if k == B.KC_FILL_NEAR and p["launches"] > 0:
            # (its work count is near pairs, not kernel evaluations: time only)
            out[B.KC_NAMES[k]] = {"ms": round(p["ms"], 2), "launches": p["launches"]}
        elif p["launches"] > 0 and p["ms"] > 0:
            r = _class_roofline(B, k, p)
            out[B.KC_NAMES[k]] = {"ms": round(p["ms"], 2), "launches": p["launches"], "bound": r["bound"],
                                  "achieved": round(r["achieved"], 3), "unit": r["unit"], "frac": round(r["frac"], 4)}
    return out


def _roofline(B, prof) -> dict:
    names = dict(enumerate(B.KC_NAMES))
    dom = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    avg_ms = p["ms"] / max(p["launches"], 1)
    roof = _class_roofline(B, dom, p)
    roof.update({"kernel": names[dom], "avg_launch_ms": avg_ms, "launches": p["launches"],
                 "traffic": measured_traffic(names[dom]),
                 "algorithmic_bytes_per_launch": p["bytes"] / max(p["launches"], 1), "traffic_unit": "bytes/launch"})
    return roof


def run_serve(args) -> int:
    """Serving mix (bem_submit / bem_poll): W warm-up requests, then a timed Poisson stream of K
    requests (one bench step = one request: mesh load, fill, nested-solve inverses, batched
    GMRES to the residual tolerance for all its plane waves), admitted by the HBM budget and
    overlapping on the device.  value = completed requests per second of wall time from the
    first timed arrival to the last completion; p50/p99 = request latency (submit to result).
    The same stream is served in each precision of --serve-precisions, the first being the
    headline (BEM_FP32 by default, then mixed and float64)."""
    import numpy as np

    import meshgen
    import paper_2106_06184_amd as B

    # restart <= 0: the library's automatic cycle length (100-1000 steps, Krylov basis <= 8 GB)
    stream = meshgen.mixed_stream(args.warmup + args.steps, rate_hz=args.serve_rate, seed=args.serve_seed)
    timed = [w for _, w in stream[args.warmup:]]
    precs = {"fp32": B.BEM_FP32, "mixed": B.BEM_MIXED, "fp64": B.BEM_FP64}
    if args.serve_profile_only:
        # only the sequential profiled pass (one host thread: for kernel traces and counters)
        prof = _profiled_pass(B, timed, args, precs[args.serve_precisions.split(",")[0]])
        print(json.dumps({"roofline": _roofline(B, prof),
                          "classes": {B.KC_NAMES[k]: v for k, v in prof.items()}}), flush=True)
        return 0
    runs = {}
    for prec_name in [p for p in args.serve_precisions.split(",") if p]:
        prec = precs[prec_name]
        log(f"serving {len(timed)} requests ({prec_name}) after {args.warmup} warm-up requests ...")
        recs, wall, comb = _serve_once(B, stream, prec, args)
        ok = [r for r in recs if r["status"] == B.BEM_OK]
        lat = [r["latency"] for r in recs if math.isfinite(r["latency"])] or [float("nan")]
        runs[prec_name] = {"value": len(ok) / wall, "wall_s": wall, "converged": len(ok), "requests": len(recs),
                           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                           "excitation_solves_per_s": sum(r["nexc"] for r in ok) / wall,
                           "combined_launches": comb[0], "combined_products": comb[1],
                           "failed": [(r["name"], r["status"]) for r in recs if r["status"] != B.BEM_OK]}
        log(f"  {prec_name}: {runs[prec_name]['value']:.3f} requests/s, p50 {runs[prec_name]['p50_s']:.2f} s, "
            f"p99 {runs[prec_name]['p99_s']:.2f} s, {len(ok)}/{len(recs)} converged")
    head = args.serve_precisions.split(",")[0]
    m, d = runs[head], runs.get("fp64", runs[head])
    log("profiled pass over the timed requests (one at a time) ...")
    prof = _profiled_pass(B, timed, args, precs[head])
    names = dict(enumerate(B.KC_NAMES))
    for k, p in prof.items():
        log(f"  {names[k]:16s} launches {p['launches']:7d}  {p['ms']:10.2f} ms  "
            f"{(p['bytes'] / p['ms'] / 1e6 if p['ms'] > 0 else 0):8.1f} GB/s  "
            f"{(p['work'] / p['ms'] / 1e9 if p['ms'] > 0 else 0):8.2f} Twork/s")
    fill_ms = sum(prof[k]["ms"] for k in (B.KC_FILL_L, B.KC_FILL_K, B.KC_FILL_NEAR, B.KC_GATHER))
    gemv_b = prof[B.KC_GEMV_F32]["bytes"] + prof[B.KC_GEMV_F64]["bytes"]
    gemv_ms = prof[B.KC_GEMV_F32]["ms"] + prof[B.KC_GEMV_F64]["ms"]
    out = {
        "metric": "solves/s + p50/p99 latency at 1e-6 relative residual (serving mix)",
        "value": m["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * m["wall_s"] / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32 storage+products, f64 refinement", "mixed": "f32+f64",
                                       "fp64": "f64"}[head], "data": "synthetic",
        "config": {"workload": "serving mix: Poisson arrivals of spheres, 1.0/0.6/0.4 ellipsoids and cubes "
                               "(cube-topology meshes of 12 n^2 triangles, T log-uniform in [320, 20000]), "
                               "eps_r ~ U[1.5, 10], k0 a ~ U[0.5, 10] redrawn below 10 mean edges per interior "
                               "wavelength, 1-64 random plane waves each; one step = one request",
                   "rate_per_s": args.serve_rate, "seed": args.serve_seed, "tol": args.tol,
                   "restart": args.restart, "precision": head, "admission": "HBM budget, 4 slots",
                   "triangles": [len(w.tri) for w in timed], "plane_waves": [len(w.khat) for w in timed]},
        "p50_s": m["p50_s"], "p99_s": m["p99_s"],
        "excitation_solves_per_s": m["excitation_solves_per_s"],
        "converged": m["converged"],
        "by_precision": {k: {f: v[f] for f in ("value", "p50_s", "p99_s", "excitation_solves_per_s", "converged",
                                               "wall_s")} for k, v in runs.items()},
        f"{head}_over_fp64": m["value"] / d["value"] if d["value"] > 0 else None,
        "fill_GBps": sum(_dense_bytes(len(w.tri)) for w in timed) / (fill_ms * 1e-3) / 1e9 if fill_ms > 0 else None,
        "matvec_frac_hbm": (gemv_b / (gemv_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS) if gemv_ms > 0 else None,
        "combined_launches": m["combined_launches"], "combined_products": m["combined_products"],
        "roofline": _roofline(B, prof),
        "kernel_classes": _kernel_classes(B, prof),
    }
    failed = {k: v["failed"] for k, v in runs.items() if v["failed"]}
    if failed:
        out["failed"] = failed
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on whole requests of the stream ...")
        out["cpu_baseline"] = serve_cpu_baseline(timed)
    print(json.dumps(out), flush=True)
    return 0 if not m["failed"] else 1


def rescale_arrivals(stream, t0: float, rate_from: float, rate_to: float):
    """The same requests in the same order arriving at `rate_to` instead of `rate_from`: every
    arrival's offset from t0 (the first timed arrival) scaled by rate_from / rate_to, which turns
    Poisson arrivals of one mean rate into those of the other."""
    scale = rate_from / rate_to
    return [(t0 + (at - t0) * scale, w) for at, w in stream]


def run_serve_sweep(args) -> int:
    """Arrival-rate sweep of the serving mix: the same W + K requests (the Poisson draws of
    `--serve-seed`) first all at once (saturated throughput: K over the wall time to the last
    completion), then at each factor of `--serve-sweep` times that rate, the arrival times
    rescaled (the same requests in the same order).  Prints one JSON line with throughput and
    request-latency percentiles per rate; no profiled pass, no CPU baseline."""
    import numpy as np

    import meshgen
    import paper_2106_06184_amd as B

    stream = meshgen.mixed_stream(args.warmup + args.steps, rate_hz=args.serve_rate, seed=args.serve_seed)
    precs = {"fp32": B.BEM_FP32, "mixed": B.BEM_MIXED, "fp64": B.BEM_FP64}
    head = args.serve_precisions.split(",")[0]
    prec = precs[head]

    def one(rescaled, label):
        log(f"serving {args.steps} requests ({head}, {label}) after {args.warmup} warm-up requests ...")
        recs, wall, _ = _serve_once(B, rescaled, prec, args)
        ok = [r for r in recs if r["status"] == B.BEM_OK]
        lat = [r["latency"] for r in recs if math.isfinite(r["latency"])] or [float("nan")]
        row = {"requests_per_s": len(ok) / wall, "wall_s": wall, "converged": len(ok), "requests": len(recs),
               "p50_s": float(np.percentile(lat, 50)), "p90_s": float(np.percentile(lat, 90)),
               "p99_s": float(np.percentile(lat, 99)),
               "excitation_solves_per_s": sum(r["nexc"] for r in ok) / wall}
        log(f"  {label}: {row['requests_per_s']:.3f} requests/s, p50 {row['p50_s']:.2f} s, "
            f"p99 {row['p99_s']:.2f} s, {len(ok)}/{len(recs)} converged")
        return row

    if args.serve_sat > 0:
        sat = args.serve_sat
        sat_row = None
    else:
        t0 = stream[args.warmup][0]
        sat_row = one([(t0, w) for _, w in stream], "all at once")
        sat = sat_row["requests_per_s"]
    t0 = stream[args.warmup][0]
    rows = []
    for f in [float(x) for x in args.serve_sweep.split(",") if x and x != "sat"]:
        rate = f * sat
        rescaled = rescale_arrivals(stream, t0, args.serve_rate, rate)
        row = one(rescaled, f"{f:.2f} x saturation = {rate:.3f} requests/s")
        row.update({"factor": f, "arrival_rate_per_s": rate})
        rows.append(row)
    timed = [w for _, w in stream[args.warmup:]]
    print(json.dumps({"sweep": "serving mix arrival rate", "precision": head, "requests": args.steps,
                      "warmup": args.warmup, "seed": args.serve_seed, "tol": args.tol,
                      "saturated_requests_per_s": sat, "saturated": sat_row, "rates": rows,
                      "triangles": [len(w.tri) for w in timed], "plane_waves": [len(w.khat) for w in timed]}),
          flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="serve",
                    help="serve (default: the serving mix), or one problem solved per step: c1, c2, "
                         "c2x256, c3, spharr, c4")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--inner", default="auto", choices=["auto", "gmres", "direct", "schur"])
    ap.add_argument("--formulation", default="sldm", choices=["sldm", "eaefie"],
                    help="sldm: the single-layer dual-mesh final system; eaefie: its comparison "
                         "formulation with the external double-layer operator")
    ap.add_argument("--exc", type=int, default=0, help="use only the first N excitations of the workload")
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--no-precond", action="store_true")
    ap.add_argument("--sweep-start", type=int, default=0,
                    help="first frequency index of a swept workload (the conductor array)")
    ap.add_argument("--no-reuse", action="store_true",
                    help="fill and invert every object separately even when objects are translated copies")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=0,
                    help="GMRES restart length (default 300; automatic when serving)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=2.0,
                    help="mean Poisson arrival rate of the serving mix, requests/s")
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--serve-profile-only", action="store_true",
                    help="run only the sequential profiled pass over the timed requests (one host thread; "
                         "for rocprofv3 kernel traces and counters of the roofline's launches)")
    ap.add_argument("--serve-precisions", default="fp32,mixed,fp64",
                    help="precisions the serving mix is run in, the first one being the headline")
    ap.add_argument("--serve-sweep", default="",
                    help="comma-separated factors of the saturated throughput: serve the mix at each of "
                         "those arrival rates (after one run with every request arriving at once) and print "
                         "the sweep instead of the benchmark line ('sat': only the run all at once)")
    ap.add_argument("--serve-sat", type=float, default=0.0,
                    help="saturated throughput (requests/s) for --serve-sweep instead of measuring it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU layout is a "
              f"design note, not a run.", file=sys.stderr)
        return 2
    if args.workload == "serve":
        return run_serve_sweep(args) if args.serve_sweep else run_serve(args)

    import numpy as np
    import torch

    import paper_2106_06184_amd as B

    w = workload(args.workload)
    prec = B.BEM_MIXED if args.precision == "mixed" else B.BEM_FP64
    inner = {"auto": B.BEM_INNER_AUTO, "gmres": B.BEM_INNER_GMRES, "direct": B.BEM_INNER_DIRECT,
             "schur": B.BEM_INNER_SCHUR}[args.inner]
    precond = 0 if args.no_precond else 1
    form = B.BEM_FORM_EAEFIE if args.formulation == "eaefie" else B.BEM_FORM_SLDM
    ctx = B.bem_create(0)
    khat, pol = (w.khat[:args.exc], w.pol[:args.exc]) if args.exc > 0 else (w.khat, w.pol)
    port = getattr(w, "port", None)
    exc = B.delta_gaps([port]) if port is not None else B.plane_waves(khat, pol)
    n_exc = 1 if port is not None else len(khat)
    # a frequency sweep (conductor array): step i solves the sweep's frequency i (cyclically)
    freqs = list(getattr(w, "freqs", [w.freq_hz]))
    nstep = [args.sweep_start]
    if args.restart <= 0:
        args.restart = 300
    opts = B.solve_opts(tol=args.tol, restart=args.restart, maxit=args.maxit)

    phases = {"mesh_load": 0.0, "assemble": 0.0, "solve": 0.0, "release": 0.0}

    def step():
        freq = freqs[nstep[0] % len(freqs)]
        nstep[0] += 1
        t0 = time.perf_counter()
        mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
        info = B.bem_mesh_info(ctx, mesh)
        t1 = time.perf_counter()
        op = B.bem_assemble(ctx, mesh, B.make_problem(freq, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg,
                                                      mu_bg=w.mu_bg, precision=prec, inner_mode=inner,
                                                      precond=precond, formulation=form, reuse=not args.no_reuse))
        t2 = time.perf_counter()
        rc, H, E, rho, si = B.bem_solve(ctx, op, exc, opts, info["n_edge"], info["n_tri"])
        t3 = time.perf_counter()
        st = B.bem_op_stats_get(ctx, op)
        B.bem_release(ctx, op)
        B.bem_release(ctx, mesh)
        t4 = time.perf_counter()
        for k, dt in zip(phases, (t1 - t0, t2 - t1, t3 - t2, t4 - t3)):
            phases[k] += dt
        if rc != B.BEM_OK or not (si.rel_residual <= args.tol):
            raise RuntimeError(f"solve failed at {freq:.4g} Hz: status {rc}, residual {si.rel_residual:.3e}")
        return info, si, st

    for i in range(args.warmup):
        info, si, st = step()
        log(f"warmup {i}: outer {si.outer_iters} res {si.rel_residual:.2e} fill {st['fill_seconds']*1e3:.1f} ms "
            f"solve {si.seconds:.3f} s")
    B.bem_profile_enable(True)
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        info, si, st = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        log(f"step {i} ({freqs[(nstep[0] - 1) % len(freqs)]:.4g} Hz): {lat[-1]:.3f} s, outer {si.outer_iters}, "
            f"refine {si.refine_steps}, "
            f"products {si.n_products}, res {si.rel_residual:.2e}, fill {st['fill_seconds']*1e3:.1f} ms")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    log("  phases per step (host wall clock, includes warm-up): " +
        ", ".join(f"{k} {1e3 * v / (args.steps + args.warmup):.1f} ms" for k, v in phases.items()))
    prof = {k: B.bem_profile_read(k) for k in range(len(B.KC_NAMES))}
    B.bem_profile_enable(False)
    names = dict(enumerate(B.KC_NAMES))
    for k, p in prof.items():
        log(f"  {names[k]:16s} launches {p['launches']:7d}  {p['ms']:10.2f} ms  "
            f"{(p['bytes'] / p['ms'] / 1e6 if p['ms'] > 0 else 0):8.1f} GB/s  "
            f"{(p['work'] / p['ms'] / 1e9 if p['ms'] > 0 else 0):8.2f} Twork/s")
    dom = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    avg_ms = p["ms"] / max(p["launches"], 1)
    if dom in (B.KC_GEMV_F64, B.KC_GEMV_F32, B.KC_GATHER):
        achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": None}
    elif dom == B.KC_GEMM_F32:
        achieved = p["work"] / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None}
    elif dom in (B.KC_DENSE_INV, B.KC_GEMM_F64):
        achieved = p["work"] / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": None}
    else:
        # fill: about 64 float64 vector operations per Green's-function evaluation
        achieved = p["work"] * 64 / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None}
    roof.update({"kernel": names[dom], "avg_launch_ms": avg_ms, "launches": p["launches"]})
    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated on a plain
    # copy) beside the algorithmic bytes per launch
    roof["traffic"] = measured_traffic(names[dom])
    roof["algorithmic_bytes_per_launch"] = p["bytes"] / max(p["launches"], 1)
    roof["traffic_unit"] = "bytes/launch"
    # single-excitation products of both precisions together
    gb = prof[B.KC_GEMV_F32]["bytes"] + prof[B.KC_GEMV_F64]["bytes"]
    gms = prof[B.KC_GEMV_F32]["ms"] + prof[B.KC_GEMV_F64]["ms"]
    matvec_frac = (gb / (gms * 1e-3) / 1e9 / HBM_PEAK_GBPS) if gms > 0 else None
    lat_sorted = sorted(lat)
    p50 = float(np.percentile(lat_sorted, 50))
    p99 = float(np.percentile(lat_sorted, 99))
    value = args.steps * n_exc / total
    out = {
        "metric": "solves/s at 1e-6 relative residual (full fill + solve per step)",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if prec == B.BEM_MIXED else "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_tri": info["n_tri"], "n_unknowns": info["n_unknowns"],
                   "excitations": n_exc, "tol": args.tol, "restart": args.restart, "precision": args.precision,
                   "inner": args.inner, "precond": bool(precond), "formulation": args.formulation, "frequencies": len(freqs),
                   "reuse_repeated_objects": not args.no_reuse, "interiors_filled": int(st["interiors_filled"])},
        "p50_s": p50, "p99_s": p99,
        "fill_GBps": st["fill_bytes"] / st["fill_seconds"] / 1e9,
        "fill_ms": st["fill_seconds"] * 1e3,
        "matvec_frac_hbm": matvec_frac,
        "roofline": roof,
    }
    B.bem_destroy(ctx)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
