"""Benchmark: solved DoF/s of the mixed-precision iterative-refinement solve
(FP64 refinement, FP16 V-cycle) against the FP64 solve on the same GPU, on the
3-D 511^3 Poisson problem with f = 14 pi^2 sin(pi x) sin(2 pi y) sin(3 pi z)
plus 1e-3 uniform noise (9 levels, V(2,2), omega = 0.8, rel. residual 1e-10).

One step = one complete solve (every kernel of the refinement loop and the
V-cycle) from u = 0 with b resident in HBM.  Prints one JSON line on stdout;
progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(solver, bt, u, steps, warmup, torch):
    for _ in range(warmup):
        solver.solve(bt, u)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    results = []
    start.record()
    for _ in range(steps):
        _, r = solver.solve(bt, u)
        results.append(r)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps, results


# the sources a kernel is built from: a traffic summary holds for them as hashed
KERNEL_SOURCES = {"ir_update": ("mg_kernels.hip", "mg_device.h"),
                  "sweep_update": ("mg_sweep_update.hip", "mg_device.h"),
                  "sweep_update_defer": ("mg_sweep_update.hip", "mg_device.h")}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2007_07539_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when that summary covers another kernel or older kernel sources."""
    if kernel not in KERNEL_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", f"{kernel}_poisson3d_511_f16_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", " ", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("traffic_kernel") != kernel or fields.get("source_sha256_16") != kernel_source_hash(kernel):
        return None
    return float(fields["traffic_bytes_per_launch"])


def kernel_table(profs, level=0):
    """Aggregate profiled refinement steps (one step's list, or a list of
    them) by kernel name on one level: launches, total time and bytes, and the
    mean launch duration."""
    if profs and isinstance(profs[0], tuple):
        profs = [profs]
    agg = {}
    for name, lvl, ms, by in (rec for prof in profs for rec in prof):
        if lvl != level:
            continue
        a = agg.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0})
        a["launches"] += 1
        a["ms"] += ms
        a["bytes"] += by
    for a in agg.values():
        a["avg_ms"] = a["ms"] / a["launches"]
        a["GBps"] = a["bytes"] / (a["ms"] * 1e-3) / 1e9 if a["ms"] > 0 else 0.0
    return agg


def profiled_steps(s, k=5):
    """k refinement steps run eagerly with every launch timed (HIP events on
    the solver's stream), after the timed solves."""
    return [s.profile_step() for _ in range(k)]


def bandwidth_ceiling(torch, mgir, reps=5):
    """Best HBM rate (GB/s, event-timed) of one streaming launch per access
    mix over a range of grid sizes: copy, read and write of 1 GiB, and the
    refinement update's mix (two FP64 arrays read and written, two FP16 arrays
    read; 36 bytes per element over 2^27 elements)."""
    dev = torch.device("cuda:0")
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ru = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    cb = torch.ones(2 * n, dtype=torch.float16, device=dev)
    out = {"metric": "streaming HBM bandwidth ceiling", "unit": "GB/s", "peak": 8000.0}
    for name, kind, bytes_moved in (("copy", 0, 2 * 8 * n), ("read", 1, 8 * n), ("write", 2, 8 * n),
                                    ("update_mix", 3, 36 * n), ("copy_nt", 4, 2 * 8 * n), ("read_nt", 5, 8 * n),
                                    ("update_mix_nt", 6, 36 * n), ("update_mix_nt_store", 7, 36 * n)):
        best = 0.0
        for blocks in (1024, 2048, 4096, 8192, 16384, 32768):
            a, b = (ru, cb) if kind in (3, 6, 7) else (dst, src)
            mgir.bandwidth_probe(a, b, kind, blocks)
            torch.cuda.synchronize()
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mgir.bandwidth_probe(a, b, kind, blocks)
                e1.record()
                torch.cuda.synchronize()
                best = max(best, bytes_moved / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        out[name] = round(best, 1)
        log(f"[ceiling] {name}: {best:.0f} GB/s")
    del src, dst, ru, cb
    torch.cuda.empty_cache()
    out["size_sweep"] = bandwidth_size_sweep(torch, mgir, reps)
    return out


def bandwidth_size_sweep(torch, mgir, reps=5):
    """Copy and read rates (GB/s, best launch shape, event-timed) of one
    streaming launch over vectors of 1 MiB to 4 GiB: the analogue of the
    paper's vector-length sweep of AXPY-like kernels (Section 8.2).  Small
    vectors expose launch latency and the caches (the 256 MB Infinity Cache
    holds the vectors up to about 128 MiB), large ones the HBM rate."""
    dev = torch.device("cuda:0")
    rows = []
    for lg in range(20, 33):
        nbytes = 1 << lg
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        row = {"bytes": nbytes}
        for name, kind, moved in (("copy", 0, 2 * nbytes), ("read", 1, nbytes)):
            best_ms = 1e30
            for blocks in (256, 1024, 4096, 16384):
                if blocks * 256 * 16 > 4 * nbytes and blocks > 256:
                    continue
                mgir.bandwidth_probe(dst, src, kind, blocks)
                torch.cuda.synchronize()
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    mgir.bandwidth_probe(dst, src, kind, blocks)
                    e1.record()
                    torch.cuda.synchronize()
                    best_ms = min(best_ms, e0.elapsed_time(e1))
            row[name] = round(moved / (best_ms * 1e-3) / 1e9, 1)
            row[name + "_us"] = round(best_ms * 1e3, 2)
        log(f"[ceiling] {nbytes >> 20} MiB: copy {row['copy']:.0f} GB/s, read {row['read']:.0f} GB/s")
        rows.append(row)
        del src, dst
        torch.cuda.empty_cache()
    return rows


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def solve_maps(torch, mgir, W, oracle, dev, dim, n, b, maps, steps, tune, defer=0):
    """Time the solve of one problem under several precision maps (the FP64
    map without residual scaling, the others with it) and check each result
    with the oracle: its FP64 relative residual ||b - A u||_2 / ||b||_2, and
    ||u - u_f64||_inf / ||u_f64||_inf against the FP64 map's solution."""
    bt = torch.from_numpy(b).to(dev)
    L = W.levels_for(n)
    out, u64 = {}, None
    nb = oracle.norm2(b)
    for name in maps:
        log(f"[bench] {dim}-D n={n} map {name}")
        kw = dict(residual_scaling=name != "f64", autotune=tune and dim == 3, device=dev)
        if name != "f64" and defer and dim == 3:
            kw["defer_update"] = defer
        s = mgir.Solver(dim, n, W.precision_map(name, L), **kw)
        u = torch.zeros_like(bt)
        ms, res = timed_solves(s, bt, u, steps, 1, torch)
        r = res[-1]
        uh = u.cpu().numpy()
        e = {"ms": round(ms, 3), "dof_per_s": n**dim / (ms * 1e-3), "iterations": r.iterations,
             "status": r.status, "rel_residual_gpu": r.rel_residual,
             "rel_residual_oracle": oracle.norm2(oracle.residual(b, uh)) / nb,
             "map": W.precision_map(name, L)}
        if name == "f64":
            u64 = uh
        elif u64 is not None:
            e["err_vs_f64"] = float(np.abs(uh - u64).max() / np.abs(u64).max())
            e["speedup_vs_f64"] = out["f64"]["ms"] / ms
        out[name] = e
        del s, u, uh
        torch.cuda.empty_cache()
    del bt
    return out, u64


def config_sweep(torch, mgir, W, oracle, dev, steps, tune, defer, cfg3=None):
    """The benchmark configurations other than the headline: the 2-D 255^2
    sine in FP64 (against the closed-form discrete solution and the oracle's
    own solve), 255^3 uniform noise FP64 vs FP16, and every precision map of
    the 511^3 problem (cfg3: results already measured there, or None)."""
    res = {}
    n = 255
    b = W.poisson2d_sine_rhs(n)
    e, u64 = solve_maps(torch, mgir, W, oracle, dev, 2, n, b, ["f64"], steps, tune)
    h = 1.0 / (n + 1)
    amp = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2   # discrete solution of the eigenmode
    uh = amp * W.sine_mode(2, n, (1, 1))
    o = oracle.ir_solve(b, residual_scaling=False, recursive_residual=True)
    e["f64"]["err_vs_discrete_closed_form"] = float(np.abs(u64 - uh).max() / np.abs(uh).max())
    e["f64"]["err_vs_oracle_solve"] = float(np.abs(u64 - o.u).max() / np.abs(o.u).max())
    e["f64"]["oracle_iterations"] = o.iterations
    res["poisson2d_255_sine_f64"] = e
    b = W.uniform_rhs(3, n, seed=2)
    res["poisson3d_255_uniform"], _ = solve_maps(torch, mgir, W, oracle, dev, 3, n, b, ["f64", "f16"], steps, tune,
                                                 defer)
    if cfg3 is not None:
        res["poisson3d_511_sine_noise"] = cfg3
    return res


def batched_shapes(mgir, s, ns):
    """The launch shapes of a batched handle per level pitch (every level of one
    pitch and format shares them once tuned): stencil {V, zc, bs, xcd, ty},
    restriction {V, tyc, zcc, pipe}."""
    out = {}
    for i, n in enumerate(ns):
        m = int(n + 1).bit_length() - 1
        for l in range(m - 1):
            key = f"P{(n + 1) >> l}"
            if key not in out:
                out[key] = {"stencil": s.get_shape(i, l, mgir.SHAPE_SWEEP, 5),
                            "restrict": s.get_shape(i, l, mgir.SHAPE_RESTRICT)}
    return out


def extra_workloads(torch, mgir, W, dev, steps, bt=None, n=511, ms64=None, tune=True, defer=0):
    """Throughput of the batched and many-right-hand-side solves (FP16 V-cycles
    and the FP64 solve of the same problems), and the paper's other precision
    variants on the main problem, each with inputs resident in HBM.  Maps with
    a narrow finest level postpone the solution update over `defer` steps, as
    the headline solve does."""
    res = {}
    if bt is not None:
        # Table 2's variants beside the main FP16 map: all-FP16 including the
        # base (H_MG), FP16 -> FP32 -> FP64 (HSD) and FP64 -> FP32 -> FP16 with
        # the residual rescaled into the FP16 levels (DSH)
        L = W.levels_for(n)
        entry = {}
        dk = {"defer_update": defer} if defer else {}
        for name, kw in (("h_mg", dk), ("hsd", dk), ("dsh", {"rescale_half": True})):
            log(f"[bench] variant {name} at {n}^3")
            s = mgir.Solver(3, n, W.precision_map(name, L), device=dev, autotune=tune, **kw)
            u0 = torch.zeros_like(bt)
            s.solve(bt, u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, r = s.solve(bt, u0)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            entry[name] = {"ms": ms, "iterations": r.iterations, "rel_residual": r.rel_residual,
                           "status": r.status, "rescale_half": name == "dsh", "defer_update": kw.get("defer_update", 0),
                           "map": W.precision_map(name, L)}
            if ms64:
                entry[name]["speedup_vs_f64"] = ms64 / ms
            del s
            torch.cuda.empty_cache()
        res[f"variants_{n}"] = entry

        # the paper's test axes: manufactured solutions k = 1, 20, 400 from a
        # random initial guess in [0, 1] (Section 6), FP16 map against FP64
        u0 = torch.from_numpy(W.random_initial_guess(3, n, seed=11)).to(dev)
        solvers = {"f16": mgir.Solver(3, n, W.precision_map("f16", L), device=dev, autotune=tune,
                                      use_initial_guess=True, **dk),
                   "f64": mgir.Solver(3, n, W.precision_map("f64", L), residual_scaling=False, device=dev,
                                      autotune=tune, use_initial_guess=True)}
        entry = {}
        for k in (1, 20, 400):
            bk = torch.from_numpy(W.manufactured_rhs(3, n, k)).to(dev)
            e = {}
            for name, s in solvers.items():
                log(f"[bench] axis k={k}, map {name}")
                u = u0.clone()
                s.solve(bk, u)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    u.copy_(u0)
                    _, r = s.solve(bk, u)
                torch.cuda.synchronize()
                e[name] = {"ms": (time.perf_counter() - t0) / steps * 1e3, "iterations": r.iterations,
                           "rel_residual": r.rel_residual, "status": r.status}
            e["speedup_f16_vs_f64"] = e["f64"]["ms"] / e["f16"]["ms"]
            entry[f"k{k}"] = e
            del bk
        del solvers, u0
        torch.cuda.empty_cache()
        res[f"axes_{n}_random_u0"] = entry

        # several V-cycles per refinement step (the inner iteration the paper's
        # conclusion points to): fewer FP64 updates per solve
        entry = {}
        for name, m in (("f16", 2), ("f16", 3), ("f64", 2)):
            log(f"[bench] {m} V-cycles per step, map {name}")
            s = mgir.Solver(3, n, W.precision_map(name, L), residual_scaling=name != "f64", device=dev,
                            autotune=tune, cycles_per_step=m, **(dk if name != "f64" else {}))
            u0 = torch.zeros_like(bt)
            s.solve(bt, u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, r = s.solve(bt, u0)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            entry[f"{name}_m{m}"] = {"ms": ms, "steps": r.iterations, "v_cycles": r.iterations * m,
                                     "rel_residual": r.rel_residual, "status": r.status}
            if ms64:
                entry[f"{name}_m{m}"]["speedup_vs_f64_m1"] = ms64 / ms
            del s
            torch.cuda.empty_cache()
        res[f"cycles_per_step_{n}"] = entry

        # partial hierarchies ending on a multi-point base level solved by CG
        # to 1e-4 relative to the base right-hand side (the paper's 1e-4 holds
        # for residuals scaled to norm one; its grids coarsen to such a base)
        entry = {}
        for name, nl in (("f16", L - 3), ("f64", L - 3), ("f16", L - 2)):
            nb = (n + 1) // 2 ** (nl - 1) - 1
            log(f"[bench] {nl} levels, CG on {nb}^3, map {name}")
            s = mgir.Solver(3, n, W.precision_map(name, nl), residual_scaling=name != "f64", device=dev,
                            autotune=tune, nlevels=nl, **(dk if name != "f64" else {}))
            u0 = torch.zeros_like(bt)
            s.solve(bt, u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, r = s.solve(bt, u0)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            entry[f"{name}_base{nb}"] = {"ms": ms, "levels": nl, "iterations": r.iterations,
                                         "rel_residual": r.rel_residual, "status": r.status}
            del s
            torch.cuda.empty_cache()
        res[f"cg_base_{n}"] = entry

        # Q1 finite elements (the paper's discretisation, Section 5) on the
        # main grid and on the paper's own meshes n = c 2^k - 1 (Section 6),
        # whose hierarchies end on a (c-1)^D base solved by CG
        entry = {}
        for dim, nq in [(3, n)] + [(3, g) for g in W.paper_grid_sizes(3)] + [(2, W.paper_grid_sizes(2)[-1])]:
            Lq = mgir.full_levels(nq)
            bq = torch.from_numpy(W.q1_load_vector(dim, nq, seed=12)).to(dev)
            e = {"dim": dim, "n": nq, "levels": Lq, "dof": float(nq**dim)}
            for name in ("f16", "f64"):
                log(f"[bench] Q1 {dim}-D n={nq}, map {name}")
                s = mgir.Solver(dim, nq, W.precision_map(name, Lq), disc="q1", residual_scaling=name != "f64",
                                device=dev, autotune=tune, **(dk if name != "f64" else {}))
                q1sh = [s.get_shape(l, k, 3 if k == mgir.SHAPE_RESTRICT else 2) for l in range(s.nlevels - 1)
                        for k in (mgir.SHAPE_SWEEP, mgir.SHAPE_RESTRICT, mgir.SHAPE_UPDATE)[: 3 if l == 0 else 2]
                        if s.get_shape(l, mgir.SHAPE_SWEEP) != [0, 0]]
                u0 = torch.zeros_like(bq)
                s.solve(bq, u0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    _, r = s.solve(bq, u0)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / steps * 1e3
                e[name] = {"ms": ms, "dof_per_s": nq**dim / ms * 1e3, "iterations": r.iterations,
                           "rel_residual": r.rel_residual, "status": r.status,
                           "defer_update": dk.get("defer_update", 0) if name != "f64" else 0,
                           "autotune": bool(tune), "lds_shapes": q1sh}
                del s, u0
                torch.cuda.empty_cache()
            e["speedup_f16_vs_f64"] = e["f64"]["ms"] / e["f16"]["ms"]
            entry[f"{dim}d_{nq}"] = e
            del bq
        res["q1_fem"] = entry

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    ns, rhs = W.batched_instances()
    dof = float(sum(n**3 for n in ns))
    bs = [torch.from_numpy(r).to(dev) for r in rhs]
    us = [torch.zeros_like(b) for b in bs]
    entry = {"instances": len(ns), "sizes": {str(n): ns.count(n) for n in sorted(set(ns))}, "dof": dof,
             "autotune": bool(tune)}
    for name, scaling in (("f16", True), ("f64", False)):
        for tuned in ((False, True) if tune else (False,)):
            log(f"[bench] batched 64 instances, map {name}{', autotuned' if tuned else ''}")
            s = mgir.BatchedSolver(ns, W.precision_map(name, 8), residual_scaling=scaling, device=dev,
                                   autotune=tuned)
            sec, (_, r, st) = timed(lambda: s.solve(bs, us))
            e = {"ms": sec * 1e3, "dof_per_s": dof / sec, "status": st,
                 "max_iterations": max(x.iterations for x in r),
                 "max_rel_residual": max(x.rel_residual for x in r)}
            if tuned:
                e["untuned_ms"] = entry[name]["ms"]
                e["shapes"] = batched_shapes(mgir, s, ns)
            entry[name] = e
            del s
            torch.cuda.empty_cache()
    entry["speedup_f16_vs_f64"] = entry["f64"]["ms"] / entry["f16"]["ms"]
    res["batched_64_instances"] = entry
    del bs, us
    torch.cuda.empty_cache()

    n, k = 127, 32
    b = torch.from_numpy(W.multi_rhs(n, k, seed=5)).to(dev)
    u = torch.zeros_like(b)
    dof = float(n**3 * k)
    entry = {"n": n, "nrhs": k, "dof_x_rhs": dof, "autotune": bool(tune)}
    for name, scaling in (("f16", True), ("f64", False)):
        for tuned in ((False, True) if tune else (False,)):
            log(f"[bench] {k} right-hand sides at {n}^3, map {name}{', autotuned' if tuned else ''}")
            s = mgir.MultiSolver(n, k, W.precision_map(name, W.levels_for(n)), residual_scaling=scaling, device=dev,
                                 autotune=tuned)
            sec, (_, r, st) = timed(lambda: s.solve(b, u))
            e = {"ms": sec * 1e3, "dof_rhs_per_s": dof / sec, "status": st,
                 "max_iterations": max(x.iterations for x in r),
                 "max_rel_residual": max(x.rel_residual for x in r)}
            if tuned:
                e["untuned_ms"] = entry[name]["ms"]
                # planes per thread of the smoothing, sweeps, prolongation; coarse
                # planes per block of the restriction
                e["shapes"] = {f"level{l}": [s.get_shape(l, kk)[1] for kk in (mgir.SHAPE_SMOOTH, mgir.SHAPE_SWEEP,
                                                                               mgir.SHAPE_PROLONG)]
                               + [s.get_shape(l, mgir.SHAPE_RESTRICT)[2]]
                               for l in range(W.levels_for(n) - 1)}
            entry[name] = e
            del s
            torch.cuda.empty_cache()
    entry["speedup_f16_vs_f64"] = entry["f64"]["ms"] / entry["f16"]["ms"]
    res["many_rhs_127x32"] = entry
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=511)
    ap.add_argument("--map", default="f16")
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle IR iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run the solve of --map with --defer (for rocprofv3)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--ceiling", action="store_true",
                    help="only measure the streaming bandwidth ceilings (copy, read, write, update mix)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched-instances and many-right-hand-sides measurements")
    ap.add_argument("--defer", type=int, default=32,
                    help="also time the mixed solve with the solution update postponed over this many steps "
                         "(0: only the per-step update); the faster one is the headline")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other precision maps and workloads (2-D 255^2, 255^3, FP32/BF16/HSD at n)")
    ap.add_argument("--q1-profile-only", action="store_true",
                    help="only run Q1 finite-element solves at --n (3-D, --map levels) for rocprofv3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2007_07539_amd import mgir
    from paper_2007_07539_amd import workloads as W

    if args.ceiling:
        print(json.dumps(bandwidth_ceiling(torch, mgir)), flush=True)
        return

    if args.q1_profile_only:
        # warm-up plus --steps timed Q1 solves of the lumped load vector
        n = args.n
        dev = torch.device("cuda:0")
        bq = torch.from_numpy(W.q1_load_vector(3, n, seed=12)).to(dev)
        Lq = mgir.full_levels(n)
        s = mgir.Solver(3, n, W.precision_map(args.map, Lq), disc="q1", residual_scaling=args.map != "f64",
                        device=dev, defer_update=args.defer if args.map != "f64" else 0,
                        autotune=not args.no_autotune)
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = s.solve(bq)
            torch.cuda.synchronize()
            log(f"[bench] Q1 solve {k}: {(time.perf_counter() - t0) * 1e3:.2f} ms, {r.iterations} steps")
        return

    n = args.n
    L = W.levels_for(n)
    N = n**3
    log(f"[bench] generating RHS n={n}")
    b = W.poisson3d_sine_noise_rhs(n, seed=3)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b).to(dev)
    u = torch.zeros_like(bt)
    tune = not args.no_autotune

    def shapes_of(s):
        return {"smooth": s.get_shape(0, mgir.SHAPE_SMOOTH), "sweep": s.get_shape(0, mgir.SHAPE_SWEEP),
                "prolong": s.get_shape(0, mgir.SHAPE_PROLONG, 7), "restrict": s.get_shape(0, mgir.SHAPE_RESTRICT),
                "update": s.get_shape(0, mgir.SHAPE_UPDATE), "fused_sweep_update": s.get_shape(0, mgir.SHAPE_FUSE, 6),
                "fused_smooth_restrict": s.get_shape(0, mgir.SHAPE_FUSE_SR, 4),
                "fused_coarse_end": s.get_shape(0, mgir.SHAPE_TAIL)}

    # the mixed solve: FP16 levels, FP64 refinement; with the solution update
    # every step (Algorithm 2 as written) and postponed over --defer steps
    mixed_runs = {}
    # (profiling: one configuration, --map with --defer; the FP64 map runs
    # without residual scaling, as the baseline does)
    depths = [args.defer] if args.profile_only else [0, args.defer] if args.defer else [0]
    for depth in depths:
        log(f"[bench] setup {args.map} solver (defer_update={depth})")
        s = mgir.Solver(3, n, W.precision_map(args.map, L), residual_scaling=args.map != "f64", device=dev,
                        autotune=tune, defer_update=depth)
        ms, res = timed_solves(s, bt, u, args.steps, args.warmup, torch)
        log(f"[bench] mixed defer={depth}: {ms:.2f} ms/solve, {res[-1].iterations} it, "
            f"rel {res[-1].rel_residual:.2e}")
        mixed_runs[depth] = {"ms": ms, "res": res[-1], "shapes": shapes_of(s), "prof": profiled_steps(s),
                             "u": u.cpu().numpy() if not args.profile_only else None}
        del s
        torch.cuda.empty_cache()
    best_depth = min(mixed_runs, key=lambda d: mixed_runs[d]["ms"])
    mx = mixed_runs[best_depth]
    ms_mixed, kt = mx["ms"], kernel_table(mx["prof"])
    if args.profile_only:
        # a plain 1 GiB device copy: the reference that scales hardware traffic
        # counters (FETCH_SIZE, WRITE_SIZE) of the solver kernels to bytes
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        mgir.bandwidth_probe(dst, src, 0)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written by k_probe")
        del src, dst

    fp64_runs = {}
    if not args.profile_only:
        # the FP64 baseline (no residual scaling, Section 6) in its fastest
        # form: the autotuner keeps the fused finest-level kernels where they
        # win; the unfused form is timed beside it for reference
        for label in ("fused", "unfused"):
            log(f"[bench] setup FP64 solver ({label})")
            s = mgir.Solver(3, n, W.precision_map("f64", L), residual_scaling=False, device=dev, autotune=tune)
            if label == "unfused":
                s.set_shape(0, mgir.SHAPE_FUSE, [0])
                s.set_shape(0, mgir.SHAPE_FUSE_SR, [0])
            ms, res = timed_solves(s, bt, u, args.steps, args.warmup, torch)
            log(f"[bench] fp64 {label}: {ms:.2f} ms/solve, {res[-1].iterations} it, rel {res[-1].rel_residual:.2e}")
            fp64_runs[label] = {"ms": ms, "res": res[-1], "shapes": shapes_of(s), "prof": profiled_steps(s),
                                "u": u.cpu().numpy() if label == "fused" else None}
            del s
            torch.cuda.empty_cache()
        best64 = min(fp64_runs, key=lambda k: fp64_runs[k]["ms"])
        ms64 = fp64_runs[best64]["ms"]

    dofs_mixed = N / (ms_mixed * 1e-3)
    # dominant kernel: the finest-level kernel with the largest share of the step
    dom_name = max(kt, key=lambda k: kt[k]["ms"])
    dom = kt[dom_name]
    achieved = dom["bytes"] / dom["launches"] / (dom["avg_ms"] * 1e-3) / 1e9

    def ktab(prof):
        return {k: {"avg_ms": round(v["avg_ms"], 4), "GBps": round(v["GBps"], 1), "launches": v["launches"]}
                for k, v in kernel_table(prof).items()}

    out = {
        "metric": "solved DoF/s to rel. residual 1e-10, mixed vs FP64 on GPU; achieved HBM GB/s",
        "value": dofs_mixed,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 refinement + f16 V-cycle (f32 accumulate)" if args.map == "f16" else args.map,
        "data": "synthetic",
        "config": {"workload": f"poisson3d_{n}_sine_noise", "n": n, "levels": L, "map": args.map,
                   "cycle": "V(2,2) damped Jacobi omega=0.8", "rtol": 1e-10, "defer_update": best_depth},
        "iterations_mixed": mx["res"].iterations,
        "rel_residual_mixed": mx["res"].rel_residual,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom_name),
                     "avg_ms": dom["avg_ms"], "bytes_per_launch": dom["bytes"] / dom["launches"]},
        "kernels_finest": ktab(mx["prof"]),
        "launch_shapes_finest": mx["shapes"],
        "mixed_by_defer_update": {str(d): {"ms": r["ms"], "iterations": r["res"].iterations}
                                  for d, r in mixed_runs.items()},
        "autotune": tune,
    }
    if not args.profile_only:
        r64 = fp64_runs[best64]
        out["fp64_value"] = N / (ms64 * 1e-3)
        out["fp64_ms_per_step"] = ms64
        out["fp64_form"] = best64
        out["iterations_fp64"] = r64["res"].iterations
        out["speedup_mixed_vs_fp64"] = ms64 / ms_mixed
        out["fp64_by_form"] = {k: {"ms": v["ms"], "iterations": v["res"].iterations,
                                   "speedup_mixed_vs_this": v["ms"] / ms_mixed} for k, v in fp64_runs.items()}
        out["kernels_finest_fp64"] = ktab(r64["prof"])
        out["launch_shapes_finest_fp64"] = r64["shapes"]
        import oracle
        oracle.build()
        # every result checked by the oracle's FP64 residual, and against the
        # FP64 map's solution
        u64 = fp64_runs["fused"]["u"]
        nb = oracle.norm2(b)
        cfg3 = {}
        for name, runs in (("f64", fp64_runs["fused"]), (args.map, mx)):
            e = {"ms": round(runs["ms"], 3), "dof_per_s": N / (runs["ms"] * 1e-3), "iterations": runs["res"].iterations,
                 "status": runs["res"].status, "rel_residual_gpu": runs["res"].rel_residual,
                 "rel_residual_oracle": oracle.norm2(oracle.residual(b, runs["u"])) / nb,
                 "map": W.precision_map(name, L)}
            if name != "f64":
                e["err_vs_f64"] = float(np.abs(runs["u"] - u64).max() / np.abs(u64).max())
                e["speedup_vs_f64"] = ms64 / runs["ms"]
            cfg3[name] = e
        out["rel_residual_oracle_mixed"] = cfg3[args.map]["rel_residual_oracle"]
        out["err_vs_f64_mixed"] = cfg3[args.map]["err_vs_f64"]
        for r in list(mixed_runs.values()) + list(fp64_runs.values()):
            r["u"] = None
        if not args.no_configs:
            for name in ("f32", "bf16", "hsd"):
                if name == args.map:
                    continue
                log(f"[bench] {n}^3 map {name}")
                kw = {"defer_update": best_depth} if best_depth else {}
                s = mgir.Solver(3, n, W.precision_map(name, L), device=dev, autotune=tune, **kw)
                ms, res = timed_solves(s, bt, u, args.steps, 1, torch)
                uh = u.cpu().numpy()
                cfg3[name] = {"ms": round(ms, 3), "dof_per_s": N / (ms * 1e-3), "iterations": res[-1].iterations,
                              "status": res[-1].status, "rel_residual_gpu": res[-1].rel_residual,
                              "rel_residual_oracle": oracle.norm2(oracle.residual(b, uh)) / nb,
                              "err_vs_f64": float(np.abs(uh - u64).max() / np.abs(u64).max()),
                              "speedup_vs_f64": ms64 / ms, "map": W.precision_map(name, L)}
                del s, uh
                torch.cuda.empty_cache()
            out["configs"] = config_sweep(torch, mgir, W, oracle, dev, args.steps, tune, best_depth, cfg3)
        else:
            out["configs"] = {"poisson3d_511_sine_noise": cfg3}
        del u64
    if not args.no_extra and not args.profile_only:
        out["extra"] = extra_workloads(torch, mgir, W, dev, args.steps, bt=bt, n=n, ms64=ms64, tune=tune,
                                       defer=best_depth)
    if not args.no_cpu_baseline and not args.profile_only:
        import oracle
        oracle.build(native=True)
        k = args.cpu_iters
        log(f"[bench] oracle: {k} FP64 IR iterations at n={n} on the host (1 thread, -O3 -march=native)")
        t0 = time.perf_counter()
        o = oracle.ir_solve(b, residual_scaling=False, recursive_residual=True, max_iter=k, native=True)
        t = time.perf_counter() - t0
        iters = out["iterations_fp64"]
        out["cpu_baseline"] = {
            "value": N / (t / max(o.iterations, 1) * iters), "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"extrapolated: {o.iterations} FP64 IR iterations of the serial C oracle (gcc -O3 "
                      f"-march=native, one thread) on the same {n}^3 RHS took {t:.1f} s including the initial "
                      f"residual; scaled to the FP64 solve's {iters} iterations (a whole solve is about "
                      f"{t / max(o.iterations, 1) * iters:.0f} s)",
            "host_cpu": host_cpu_model(), "host_cpus": os.cpu_count(),
        }
        log(f"[bench] oracle: {t:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
