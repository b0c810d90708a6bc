#!/usr/bin/env python
"""Benchmark of the WCSPH time step on one MI355X.

A step is one pass of the whole path on the GPU: cell keys with migration
labels, stable radix sort, reorder, cell tables, interaction, dt reduction and
Verlet update (sph_step). The workload is the dam break with three obstacles
at dp = 0.004 m (about 1.47M particles, seeded synthetic lattice, starting at
hydrostatic rest). The state is resident in HBM before the timed region.

Prints one JSON line: whole-step pair interactions/s (value), steps/s, the
roofline of the dominant kernel (the interaction) with its duration measured
by HIP events on the step's stream, and the FP64 CPU oracle timed on the host
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 work per neighbour pair of the interaction, counted from the equations
# (mul/add/sub/sqrt/rcp = 1, fused multiply-add = 2): separation 3, r^2 5,
# r 1, 1 - q/2 2, (1-q/2)^3 2, kernel gradient factor 1, v_ij 3, v_ij.r_ij 5,
# continuity sum 2, mu 4, |mu| max 1, c_j 3, viscous term 6, pressure sum 2,
# force factor 1, three force sums 6.
FLOP_PER_PAIR = 47
# The cubic spline's gradient factor in place of Wendland's (1 - q/2, its
# cube: 4): q 1, 2 - q 1, square 1, reciprocal 1 and product 1, 4 - 3q 2.
FLOP_PER_PAIR_CUBIC = FLOP_PER_PAIR - 4 + 7
# FP32 work of one support test of a candidate j: separation 3, r^2 5.
FLOP_PER_CANDIDATE = 8
# Compulsory HBM bytes of the interaction per in-domain particle: read x, y, z,
# vx, vy, vz, rho (28) and the type (1); write ax, ay, az, drho/dt (16).
BYTES_PER_PARTICLE_INTERACT = 45
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X, packed FP32 (256 CU x 2.4 GHz)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # FMA on 64 lanes/CU/clk without packed math
PEAK_HBM_GBS = 8000.0


def _src_hash(paths) -> str:
    h = hashlib.sha256()
    for path in ([paths] if isinstance(paths, str) else paths):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_src, launches_key: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(launches_key)
    except Exception:
        return None
    if not rec or rec.get("source_sha256_16") != _src_hash(kernel_src):
        return None
    return rec.get("bytes_per_launch")


def _json_default(o):
    """numpy scalars in the JSON lines."""
    if hasattr(o, "item"):
        return o.item()
    raise TypeError(f"not JSON serialisable: {type(o).__name__}")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, seconds: float) -> dict:
    """The FP64 oracle as it stands, full steps of the same workload from its
    initial state: about ``seconds`` of wall time on all host threads (the
    reported value), then the first step again on one thread (at least one
    step, about a third of ``seconds`` at most beyond it)."""
    import oracle

    def timed(budget, min_steps):
        st = case.state
        pairs = steps = 0
        t0 = time.perf_counter()
        while steps < min_steps or (time.perf_counter() - t0 < budget and steps < 200):
            r = oracle.step(case.params, st, steps)
            st = r["state"]
            pairs += r["pairs"]
            steps += 1
        return pairs, steps, time.perf_counter() - t0

    all_threads = oracle.threads()
    pairs, steps, el = timed(seconds, 3)
    oracle.set_threads(1)
    try:
        p1, s1, e1 = timed(seconds / 3.0, 1)
    finally:
        oracle.set_threads(all_threads)
    return {"value": pairs / el, "unit": "pair interactions/s", "cores": all_threads,
            "kind": "oracle",
            "sample": f"{steps} full FP64 oracle steps of the same workload from its initial "
                      f"state ({pairs} pair interactions in {el:.2f} s; OpenMP over particles, "
                      f"{all_threads} threads)",
            "steps_per_s": steps / el, "cpu_model": _cpu_model(),
            "host_cpus": os.cpu_count(),
            "one_thread": {"value": p1 / e1, "steps": s1, "seconds": e1,
                           "steps_per_s": s1 / e1}}


def copy_probe(mib: int, reps: int) -> None:
    """A plain device-to-device copy of known size, for scaling the HBM
    counters of rocprofv3 (FETCH_SIZE / WRITE_SIZE per dispatch)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "reps": reps}), flush=True)


def machine_probe(reps: int) -> dict:
    """What this GPU reaches with the library's own build flags: an FP32 FMA
    loop (non-packed) and a 16-byte streaming copy (sph_probe_fma /
    sph_probe_copy), next to torch's device copy. Context for the roofline
    fractions, which stay quoted against the published peaks."""
    import torch
    from paper_1210_1017_amd import sph
    blocks_fma, iters = 2048, 8192
    out = torch.empty(blocks_fma * 256, dtype=torch.float32, device="cuda")
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    t_fma = timed(lambda: sph.probe_fma(out, blocks_fma, iters))
    t_copy = timed(lambda: sph.probe_copy(src, dst, 1024))
    t_torch = timed(lambda: dst.copy_(src))
    if not torch.equal(dst, src):
        raise RuntimeError("copy probe: destination differs from source")
    fma = 16.0 * iters * blocks_fma * 256 / t_fma / 1e12
    copy = 2.0 * nbytes / t_copy / 1e9
    return {"fma_tflops": fma, "fma_frac_of_nonpacked_peak": fma / PEAK_FP32_NONPACKED_TFLOPS,
            "copy_gbs": copy, "copy_frac_of_hbm_peak": copy / PEAK_HBM_GBS,
            "torch_copy_gbs": 2.0 * nbytes / t_torch / 1e9,
            "fma": f"{blocks_fma} x 256 lanes x {iters} iterations of 8 independent FP32 FMAs",
            "copy": "1 GiB read + 1 GiB written, 16-byte vectors, 4 per lane per pass, 1024 x 256 lanes",
            "reps": reps}


def variants(case, steps: int, warmup: int = 10) -> dict:
    """Steps/s and pair interactions/s of the step variants (sph_params.options)
    on the same workload, each from the initial state; the interaction phase
    (both interactions and the half step for the symplectic integrator) by
    HIP events on the step's stream."""
    import torch

    from paper_1210_1017_amd import sph
    out = {}
    n = case.n
    for name, opts in (("cubic", sph.OPTION_CUBIC), ("symplectic", sph.OPTION_SYMPLECTIC),
                       ("cubic_symplectic", sph.OPTION_CUBIC | sph.OPTION_SYMPLECTIC)):
        p = dict(case.params)
        p["options"] = opts
        ctx = sph.Context(p, n)
        a = sph.DeviceState.from_numpy(case.state, capacity=n)
        b = sph.DeviceState.empty(n)
        for s in range(warmup):
            ctx.step(a, b, n, s)
            a, b = b, a
        torch.cuda.synchronize()
        pairs0, cand0 = ctx.pair_total(), ctx.candidate_total()
        ctx.timing_begin(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(warmup, warmup + steps):
            ctx.step(a, b, n, s)
            a, b = b, a
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ph = ctx.timing_read(steps)
        ctx.timing_begin(0)
        inter = 2 if opts & sph.OPTION_SYMPLECTIC else 1
        pairs = ctx.pair_total() - pairs0
        cand = ctx.candidate_total() - cand0
        fpp = FLOP_PER_PAIR_CUBIC if opts & sph.OPTION_CUBIC else FLOP_PER_PAIR
        t_int = float(ph[:, 1].mean()) * 1e-3
        flop = fpp * pairs / steps + FLOP_PER_CANDIDATE * cand / steps
        out[name] = {"options": opts, "steps": steps, "ms_per_step": el / steps * 1e3,
                     "steps_per_s": steps / el, "pair_interactions_per_s": pairs / el,
                     "interactions_per_step": inter, "interact_phase_ms": t_int * 1e3,
                     "alu_frac_interact_phase": flop / t_int / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                     "status": ctx.status()}
        print(f"[bench] variant {name}: {out[name]}", file=sys.stderr, flush=True)
        del ctx, a, b
    return out


def _by_id(arrs: dict, ids):
    import numpy as np
    order = np.argsort(ids, kind="stable")
    return {k: v[order] for k, v in arrs.items()}


def precision_report(args) -> dict:
    """Precision variant: the same workload advanced by the plain FP32 path
    (absolute FP32 positions), the cell + offset FP32 path and the FP64 path;
    FP64 totals (mass, momentum, energy) along the run and per-quantity
    differences against the FP64 run by particle id. (The comparison of one
    cell-path step with the FP64 oracle on a 64-spacing cube of this workload
    is a GPU test.)"""
    import numpy as np
    import torch

    from paper_1210_1017_amd import cases, sph

    t0 = time.perf_counter()
    case = cases.case_c4() if args.report_case == "c4" else cases.case_c2()
    p, n = case.params, case.n
    print(f"[precision] {case.name}: {n} particles, generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    F = sph.FEATURE_CELL | sph.FEATURE_FP64
    ctx = sph.Context(p, n, F)
    t64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    # cell + offset state from the exact lattice positions
    ca, cb = sph.CellState.empty(n), sph.CellState.empty(n)
    ctx.cstate_from_positions(t64(case.pos64[:, 0]), t64(case.pos64[:, 1]), t64(case.pos64[:, 2]),
                              ca, n)
    for k in ("vx", "vy", "vz", "rho", "vxp", "vyp", "vzp", "rhop", "type", "id"):
        ca.t[k][:n].copy_(torch.from_numpy(np.ascontiguousarray(case.state[k])))
    # FP64 state from the same positions
    st64 = {k: case.state[k] for k in sph.SOA_FIELDS}
    st64["x"], st64["y"], st64["z"] = case.pos64[:, 0], case.pos64[:, 1], case.pos64[:, 2]
    da, db = sph.F64State.from_numpy(st64, capacity=n), sph.F64State.empty(n)
    # plain FP32 state (positions rounded to FP32)
    pa, pb = sph.DeviceState.from_numpy(case.state, capacity=n), sph.DeviceState.empty(n)
    del st64
    out = {"workload": case.name, "particles": n, "steps": args.report_steps,
           "fp64_steps": args.fp64_steps, "series": []}

    def plain_totals(s):
        st = {k: s.t[k][:n].double() for k in ("x", "y", "z", "vx", "vy", "vz", "rho")}
        ng = s.t["type"][:n] != cases.GHOST
        m = p["mass"]
        rho0, B = p["rho0"], p["c0"] ** 2 * p["rho0"] / 7.0
        sr = st["rho"] / rho0
        e = B * ((sr ** 6 - 1.0) / (6 * rho0) + (1.0 / st["rho"] - 1.0 / rho0))
        tot = [m * ng.sum(), m * st["vx"][ng].sum(), m * st["vy"][ng].sum(), m * st["vz"][ng].sum(),
               0.5 * m * (st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)[ng].sum(),
               m * 9.81 * st["z"][ng].sum(), m * e[ng].sum(), ng.sum()]
        return [float(v) for v in tot]

    def compare(step):
        """Per-quantity differences of the cell and plain FP32 runs against
        the FP64 run, by particle id, at the current step."""
        ref = _by_id(da.to_numpy(n), da.t["id"][:n].cpu().numpy())
        x, y, z = ctx.cstate_positions(ca, n)
        cst = ca.to_numpy(n)
        cst.update({"x": x.cpu().numpy(), "y": y.cpu().numpy(), "z": z.cpu().numpy()})
        cel = _by_id(cst, cst["id"])
        pla = _by_id(pa.to_numpy(n), pa.t["id"][:n].cpu().numpy())
        fl = ref["type"] == cases.FLUID
        errs = {"step": step}
        for name, st in (("cell", cel), ("plain", pla)):
            e = {}
            for k in ("x", "y", "z", "vx", "vy", "vz", "rho"):
                d = st[k][fl].astype(np.float64) - ref[k][fl]
                e[k] = {"rms": float(np.sqrt(np.mean(d * d))), "max": float(np.abs(d).max())}
            disp = np.sqrt(sum((ref[k][fl] - case.pos64[ref["id"][fl], i]) ** 2
                               for i, k in enumerate("xyz")))
            e["rms_displacement_fp64"] = float(np.sqrt(np.mean(disp ** 2)))
            errs[name] = e
        return errs

    ev = max(1, min(args.report_steps // 10, 250))  # a progress line at least every 250 steps
    tc = td = tp = 0.0
    for s in range(args.report_steps + 1):
        if s % ev == 0 or s == args.report_steps:
            rec = {"step": s, "cell": ctx.ctotals(ca, n).tolist(), "plain": plain_totals(pa)}
            if s <= args.fp64_steps:
                rec["fp64"] = ctx.dtotals(da, n).tolist()
            out["series"].append(rec)
            print(f"[precision] step {s}: {rec}", file=sys.stderr, flush=True)
        if s == args.fp64_steps or (s == 1000 and args.fp64_steps > 1000):
            # against the FP64 run at step 1,000 (before the flow turns chaotic)
            # and at the FP64 run's last step
            rec = compare(s)
            out.setdefault("vs_fp64_at", []).append(rec)
            out.setdefault("vs_fp64", rec)
            print(f"[precision] vs FP64 at step {s}: {rec}", file=sys.stderr, flush=True)
        if s == args.report_steps:
            break
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.cstep(ca, cb, n, s)
        ca, cb = cb, ca
        torch.cuda.synchronize()
        b = time.perf_counter()
        ctx.step(pa, pb, n, s)
        pa, pb = pb, pa
        torch.cuda.synchronize()
        c = time.perf_counter()
        tc += b - a
        tp += c - b
        if s < args.fp64_steps:
            ctx.dstep(da, db, n, s)
            da, db = db, da
            torch.cuda.synchronize()
            td += time.perf_counter() - c
    out["ms_per_step"] = {"cell": tc / args.report_steps * 1e3, "plain": tp / args.report_steps * 1e3,
                          "fp64": td / max(args.fp64_steps, 1) * 1e3}
    return out


def slab_bench(args) -> dict:
    """One GPU's sub-domain at its real shape: slab 1 of a 4-slab x
    decomposition of the dam break at dp = 1.3 mm (8,000,525 fluid particles,
    walls, ghost strips of width 2h on both x faces), in developed flow
    (v ~ U(-0.5, 0.5) m/s, rho x (1 +- 0.5 %)). Before each step a migration
    injector stands in for the neighbouring sub-domains (Sec. 4.2): 0.25 % of
    the fluid per face (20,001 particles), drawn with PCG64(5 + step) from the
    fluid of the layer next to the face, is moved across the face by U(0, dp);
    after the step (sort with migration labels, interaction, update) the
    outgoing ranges of the sort (Sec. 4.3) are wrapped back in through the
    opposite face (x -/+ the slab width), so the particle count is exactly
    conserved, which is asserted every step. Kernel time per step comes from
    HIP events on the step's stream; the injector runs between steps and is
    timed apart from them."""
    import numpy as np
    import torch

    from paper_1210_1017_amd import cases, migration, sph

    t0 = time.perf_counter()
    case = cases.perturb(cases.slab_c3(), 6)
    p, n = case.params, case.n
    cnt = case.counts()
    print(f"[slab] {case.name}: {n} particles {cnt}, generated in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    nmig = int(round(0.0025 * cnt["fluid"]))
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)

    books = {"migrated_out": 0, "wrapped": 0}

    def run(k, s0):
        tin = 0.0
        for s in range(s0, s0 + k):
            t1 = time.perf_counter()
            books["migrated_out"] += migration.inject(a_b[0], n, p, s, nmig)
            torch.cuda.synchronize()
            tin += time.perf_counter() - t1
            ctx.step(a_b[0], a_b[1], n, s)
            c = ctx.counts()  # synchronises
            t1 = time.perf_counter()
            if sum(c["n_label"]) != n or c["n_label"][3] != 0:
                raise RuntimeError(f"step {s}: particle count not conserved: {c['n_label']}")
            if c["n_label"][1] < nmig or c["n_label"][2] < nmig:
                raise RuntimeError(f"step {s}: injected migrants missing: {c['n_label']}")
            books["wrapped"] += migration.wrap(a_b[1], c, p)
            torch.cuda.synchronize()
            tin += time.perf_counter() - t1
            a_b.reverse()
        return tin

    a_b = [a, b]
    run(args.warmup, 0)
    pairs0, cand0 = ctx.pair_total(), ctx.candidate_total()
    ctx.timing_begin(args.steps)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    t_inj = run(args.steps, args.warmup)
    t_wall = time.perf_counter() - t_wall
    ph = ctx.timing_read(args.steps)
    ctx.timing_begin(0)
    pairs = ctx.pair_total() - pairs0
    cand = ctx.candidate_total() - cand0
    c = ctx.counts()
    status = ctx.status()
    movers, path = ctx.sort_stats()
    kern_ms = float(ph.sum(axis=1).mean())
    t_int = float(ph[:, 1].mean()) * 1e-3
    pairs_per_launch = pairs / args.steps
    flop = FLOP_PER_PAIR * pairs_per_launch + FLOP_PER_CANDIDATE * cand / args.steps
    achieved = flop / t_int / 1e12
    out = {"workload": case.name, "particles": n, "fluid": cnt["fluid"],
           "boundary": cnt["boundary"], "ghost": cnt["ghost"], "steps": args.steps,
           "warmup": args.warmup, "migrants_per_face_per_step": nmig,
           "ms_per_step_kernels": kern_ms, "steps_per_s_kernels": 1e3 / kern_ms,
           "pair_interactions_per_s_kernels": pairs / (ph.sum() * 1e-3),
           "phase_ms": {"sort": float(ph[:, 0].mean()), "interact": float(ph[:, 1].mean()),
                        "dt_update": float(ph[:, 2].mean())},
           "wall_ms_per_step_with_injector": t_wall / args.steps * 1e3,
           "injector_ms_per_step": t_inj / args.steps * 1e3,
           "interact": {"bound": "alu", "achieved_tflops": achieved,
                        "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                        "frac_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                        "pairs_per_launch": pairs_per_launch,
                        "candidates_per_launch": cand / args.steps,
                        "hbm_gbs_algorithmic":
                            BYTES_PER_PARTICLE_INTERACT * c["n_label"][0] / t_int / 1e9},
           "last_counts": c, "migrated_out": books["migrated_out"], "wrapped": books["wrapped"],
           "dt_last": float(ctx.dt()), "status": int(status),
           "sort_path": {"movers_last_step": movers,
                         "path": ("radix", "merge", "merge_mover_passes")[path]}}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time of the CPU-oracle baseline (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter scaling) and exit")
    ap.add_argument("--precision-report", action="store_true",
                    help="run the precision-variant report (cell + offset and FP64 paths) and exit")
    ap.add_argument("--report-case", default="c4", choices=["c4", "c2"])
    ap.add_argument("--slab", action="store_true",
                    help="time one GPU's slab of a 4-slab decomposition (8.8M particles) with "
                         "the per-step migration injector, print its JSON line and exit")
    ap.add_argument("--report-steps", type=int, default=10000)
    ap.add_argument("--fp64-steps", type=int, default=10000)
    ap.add_argument("--variant-steps", type=int, default=200,
                    help="timed steps of each step variant (cubic kernel, symplectic "
                         "integrator) added to the JSON line (0: skip)")
    ap.add_argument("--probe-reps", type=int, default=10,
                    help="repeats of the machine probes (FMA loop, streaming copy) added "
                         "to the JSON line (0: skip)")
    ap.add_argument("--surrogate-steps", type=int, default=1000,
                    help="steps of the surrogate-vs-plain comparison added to the JSON line "
                         "when trained weights are present (0: skip)")
    args = ap.parse_args()
    if args.precision_report:
        print(json.dumps(precision_report(args)), flush=True)
        return 0
    if args.copy_probe:
        copy_probe(args.copy_probe, 5)
        return 0
    if args.slab:
        print(json.dumps(slab_bench(args), default=_json_default), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the multi-GPU "
              "exchange of the method is not implemented in this package.", file=sys.stderr)
        return 2

    import torch

    from paper_1210_1017_amd import cases, sph

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    case = cases.case_c2()
    p, n = case.params, case.n
    print(f"[bench] workload {case.name}: {n} particles {case.counts()}; "
          f"warmup {args.warmup}, timed steps {args.steps}", file=sys.stderr, flush=True)
    ctx = sph.Context(p, n)
    a = sph.DeviceState.from_numpy(case.state, capacity=n)
    b = sph.DeviceState.empty(n)
    for s in range(args.warmup):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    pairs0 = ctx.pair_total()
    cand0 = ctx.candidate_total()
    ctx.timing_begin(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        ctx.step(a, b, n, s)
        a, b = b, a
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pairs = ctx.pair_total() - pairs0
    phases = ctx.timing_read(args.steps)
    cand = ctx.candidate_total() - cand0
    status = ctx.status()
    counts = ctx.counts()
    movers, merged = ctx.sort_stats()
    ctx.timing_begin(0)
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s; status {status}; counts "
          f"{counts['n_label']}", file=sys.stderr, flush=True)

    t_int = float(phases[:, 1].mean()) * 1e-3
    pairs_per_launch = pairs / args.steps
    flop = FLOP_PER_PAIR * pairs_per_launch + FLOP_PER_CANDIDATE * (cand / args.steps)
    achieved = flop / t_int / 1e12
    kernel_src = [os.path.join(ROOT, "paper_1210_1017_amd", "csrc", f)
                  for f in ("interact.hip", "sph_device.h")]
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "traffic": _traffic(kernel_src, "k_interact:c2"),
            "kernel": "k_interact", "kernel_ms": t_int * 1e3,
            "flop_per_launch": flop, "pairs_per_launch": pairs_per_launch,
            "candidates_per_launch": cand / args.steps,
            "frac_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "hbm_gbs_algorithmic": BYTES_PER_PARTICLE_INTERACT * counts["n_label"][0] / t_int / 1e9}
    out = {
        "metric": "pair interactions/s, steps/s @1M particles; surrogate speedup at \u22641% \u03c1 error",
        "value": pairs / elapsed,
        "unit": "pair interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "steps_per_s": args.steps / elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": case.name, "particles": n, "fluid": case.counts()["fluid"],
                   "boundary": case.counts()["boundary"], "dp_m": p["dp"], "h_over_dp": 1.3,
                   "kernel": "wendland_c2", "cfl": p["cfl"], "sort": "every step"},
        "phase_ms": {"sort": float(phases[:, 0].mean()), "interact": float(phases[:, 1].mean()),
                     "dt_update": float(phases[:, 2].mean())},
        "roofline": roof,
        # which way the last timed step sorted: the movers (keys changed since
        # the previous sort) merged with the rest (sorted by one block, or by
        # their own radix passes), or the full radix sort
        "sort_path": {"movers_last_step": movers, "merged_last_step": bool(merged),
                      "path": ("radix", "merge", "merge_mover_passes")[merged]},
    }
    if args.probe_reps > 0:
        out["machine"] = machine_probe(args.probe_reps)
        roof["frac_measured_fma"] = achieved / out["machine"]["fma_tflops"]
    if args.variant_steps > 0:
        out["variants"] = variants(case, args.variant_steps)
    from paper_1210_1017_amd import surrogate
    wpath = surrogate.default_weights()
    if args.surrogate_steps > 0 and os.path.exists(wpath):
        print(f"[bench] surrogate vs plain SPH, {args.surrogate_steps} steps", file=sys.stderr,
              flush=True)
        rep = surrogate.report(steps=args.surrogate_steps, weights=wpath,
                               log=lambda *m: print(*m, file=sys.stderr, flush=True))
        judged = [j["max_rel_rho"] for j in rep["judge"]]
        ser = rep["vs_plain_trajectory"]
        out["surrogate"] = {
            "workload": rep["workload"], "steps": rep["steps"],
            # steps/s ratio over the whole run; the run falls back to plain SPH
            # once a judged window exceeds 1 %, so this is not a figure at 1 %
            "speedup": rep["speedup"],
            # accumulated error against the plain trajectory from the same start
            "steps_within_1pct_of_plain_trajectory": ser["steps_within_tol"],
            "speedup_within_1pct_of_plain_trajectory":
                rep["speedup_within_tol_of_plain_trajectory"],
            "max_rel_rho_vs_plain_trajectory": [
                (q["step"], q["max_rel_rho"]) for q in ser["series"]],
            "steps_per_s": rep["surrogate_steps_per_s"],
            "plain_steps_per_s": rep["plain_steps_per_s"],
            "judge_max_rel_rho": max(judged) if judged else None,
            "judged_advances": len(judged), "advances": rep["surrogate_books"]["advances"],
            "fallback_at": rep["surrogate_books"]["fallback_at"],
            "residual": bool(rep["config"].get("residual", False)),
            "final_vs_plain": rep["final_vs_plain"],
            "persistence_final_vs_plain": rep["persistence_final_vs_plain"]}
        if "rates_only_final_vs_plain" in rep:
            out["surrogate"]["rates_only_final_vs_plain"] = rep["rates_only_final_vs_plain"]
            out["surrogate"]["rates_only_fallback_at"] = rep["rates_only_books"]["fallback_at"]
    if args.cpu_seconds > 0:
        print(f"[bench] CPU oracle baseline: ~{args.cpu_seconds:.0f} s", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
