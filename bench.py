#!/usr/bin/env python3
"""Throughput benchmark: batched GLL spectral Poisson solves to 1e-10 relative
residual, preconditioned by the p-multigrid gamma-cycle, on one MI355X.

Workload (default): 2-D deformed square, p = 128 (129 x 129 nodes),
gamma-cycle p = 128 -> 64 -> ... -> 2, FP64, mapping
x = s + a sin(pi s) sin(pi t), y = t + b sin(2 pi s) sin(pi t), a, b ~ U[0, 0.15],
16-mode Fourier right-hand side, 8-mode Dirichlet data; synthetic, seeded.

A step is one pass of the whole path over one batch of B problems already
resident in HBM: setup (geometry, line tridiagonals and their
cyclic-reduction factors on every level), Dirichlet lifting of the
right-hand side, the preconditioned Krylov solve, and the final lift.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_FP32_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--p", type=int, default=128)
    ap.add_argument("--gamma", type=int, default=3)
    ap.add_argument("--gamma3", type=int, default=1, help="gamma of the 3-D leg")
    ap.add_argument("--restriction3", choices=["interp", "transpose"], default="transpose",
                    help="R of the 3-D leg (the paper has no 3-D experiment)")
    ap.add_argument("--restriction", choices=["interp", "transpose"], default="interp",
                    help="R of Sec. 3.3: interpolation (reproduces Table 1) or P^T")
    ap.add_argument("--alpha", type=float, default=0.16)
    ap.add_argument("--smoother", choices=["fem", "gll"], default="fem")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--krylov", choices=["fgmres", "pcg", "fcg"], default="fgmres")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle CPU baseline (0 disables it)")
    ap.add_argument("--serve", type=int, default=4096, metavar="N",
                    help="requests of the served mixed 2-D/3-D stream (0 skips serving)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="paced arrival rate as a fraction of the saturated throughput")
    ap.add_argument("--mixed", type=int, default=1, help="also time the FP32-inner solve")
    ap.add_argument("--components", type=int, default=1,
                    help="also time the operator and line-solve kernels alone")
    ap.add_argument("--sweep", type=int, default=1,
                    help="also time gamma = 1, 2, 3, 7 and the R = P^T variant")
    ap.add_argument("--legs", type=int, default=1,
                    help="also time 3-D p = 64 and 2-D p = 256, FP64 and FP32 cycle")
    ap.add_argument("--legs-batch3", type=int, default=128)
    ap.add_argument("--elements", type=int, default=1,
                    help="spectral elements per axis of the headline run (profiling of the "
                         "element path; the default run and its metric use one element)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: the reference that scales the HBM
    byte counters (FETCH_SIZE, WRITE_SIZE) of the solve kernel."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                      "launches": 3}), flush=True)


def flops_per_solve(dim, p, gamma, m, iters, krylov, restart, collapsed=(), elements=1):
    """Algorithmic flop count of one solve: per level visit the operator's
    contractions and flux products, the line sweeps' cyclic reduction, the
    transfers and the vector updates; per outer iteration the FP64 operator
    and the Krylov vector work.  A level in `collapsed` (degrees) is applied
    as its dense matrix: 2 ni^2 flops per visit, and the levels below it are
    not visited.  elements = K > 1 (2-D): every level is K x K elements of
    degree p_l / K (the operator's contractions per element, the transfers'
    element blocks), the hierarchy stops at degree 2K (dense exact solve)."""
    K = elements

    def level_costs(pl):
        n1 = pl + 1
        N = n1 ** dim
        nint = (pl - 1) ** dim
        if K > 1:
            ne1 = pl // K + 1
            apply_ = K ** dim * (4 * dim * ne1 + (2 * dim * dim - dim)) * ne1 ** dim + N
            nb = K * ne1 * (pl // (2 * K) + 1)          # nonzeros of a 1-D composite transfer
            n1c = pl // 2 + 1
            transfer = 2 * nb * (n1 + n1c)
            return apply_, 11 * nint, transfer
        apply_ = (4 * dim * n1 + (2 * dim * dim - dim) + 1) * N
        cr = 11 * nint
        n1c = pl // 2 + 1
        if dim == 2:
            transfer = 2 * n1 * n1c * (n1 + n1c)
        else:
            transfer = 2 * (n1**3 * n1c + n1**2 * n1c**2 + n1 * n1c**3)
        return apply_, cr, transfer

    levels = []
    pl = p
    while pl >= 2 * K:
        levels.append(pl)
        pl //= 2
    if K > 1:
        collapsed = tuple(collapsed) + (2 * K,)
    cycle = 0.0
    for depth, pl in enumerate(levels):
        visits = gamma ** depth
        if pl in collapsed:
            cycle += visits * 2 * (pl - 1) ** (2 * dim)
            break
        if pl == 2:
            cycle += visits * 1
            continue
        a, c, t = level_costs(pl)
        sweeps = dim * m * (1 + gamma)
        cycle += visits * ((sweeps - 1 + gamma) * a + sweeps * c + 2 * gamma * t)
    a_f, _, _ = level_costs(p)
    N = (p + 1) ** dim
    total = 0.0
    if krylov == "fgmres":
        j = 0
        restarts = 1
        for _ in range(iters):
            total += cycle + a_f + 4 * (j + 1) * N + 3 * N
            j += 1
            if j == restart:
                j = 0
                restarts += 1
        total += restarts * (a_f + 4 * N) + iters * 2 * N
    else:
        total += (iters + 1) * (cycle + a_f + 12 * N)
    return total


def make_problems(dim, B, seed0=0):
    from paper_2504_10710_amd import inputs
    make = inputs.config2 if dim == 2 else inputs.config3
    return [make(seed0 + s) for s in range(B)]


def run_batch(args, prec_name, dim=2, p=None, B=None, gamma=None, restriction=None,
              steps=None, warmup=None, keep=0, restart=None, tag="", elements=1):
    """Time `steps` whole-path steps of one batch; returns the measurements.
    keep > 0 also returns the solutions of the first `keep` problems."""
    import numpy as np
    import torch

    from paper_2504_10710_amd import inputs, pmg

    dev = torch.device("cuda:0")
    B = args.batch if B is None else B
    p = args.p if p is None else p
    gamma = args.gamma if gamma is None else gamma
    restriction = args.restriction if restriction is None else restriction
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    restart = (args.restart if dim == 2 else 20) if restart is None else restart
    smoother = pmg.PMG_SMOOTHER_FEM if args.smoother == "fem" else pmg.PMG_SMOOTHER_GLL
    prec = pmg.PMG_F32 if prec_name == "f32" else pmg.PMG_F64
    krylov = {"fgmres": pmg.PMG_FGMRES, "pcg": pmg.PMG_PCG, "fcg": pmg.PMG_FCG}[args.krylov]
    rst = pmg.PMG_RESTRICT_INTERP if restriction == "interp" else pmg.PMG_RESTRICT_TRANSPOSE
    desc = pmg.make_desc(dim=dim, p_fine=p, batch=B, gamma=gamma, m=1, alpha=args.alpha,
                         smoother=smoother, inner_prec=prec, krylov=krylov,
                         restart=restart, max_iter=600, rtol=args.rtol, restriction=rst,
                         elements=elements)
    label = f"{tag or prec_name} {dim}-D p={p} gamma={gamma} R={restriction}"
    if elements > 1:
        label += f" {elements}x{elements} elements"

    # ---- synthetic inputs (seeded), resident in HBM before timing
    t0 = time.time()
    probs = make_problems(dim, B)
    K = elements
    # levels below degree 2K are absent for K elements per axis (no coordinates)
    l0 = pmg.pmg_first_level(desc)
    ps = inputs.halving_degrees(p, 2 * K)
    coords = [None] * l0

    def nodes(q):   # composite node grid of level degree q (K elements of degree q / K)
        return inputs.composite_nodes(pmg.pmg_gll(q // K)[0], K) if K > 1 else pmg.pmg_gll(q)[0]
    for q in ps:
        xi = nodes(q)
        coords.append(torch.from_numpy(np.stack([pr.coords(xi) for pr in probs])).to(dev))
    xi = nodes(p)
    Xf = [pr.coords(xi) for pr in probs]
    f = torch.from_numpy(np.stack([pr.f(x) for pr, x in zip(probs, Xf)])).to(dev)
    g = torch.from_numpy(np.stack([pr.g(x) for pr, x in zip(probs, Xf)])).to(dev)
    ws = torch.empty(pmg.pmg_workspace_bytes(desc), dtype=torch.uint8, device=dev)
    info = torch.empty(B * pmg.INFO_BYTES, dtype=torch.uint8, device=dev)
    b = torch.empty_like(f)
    x = torch.empty_like(f)
    u = torch.empty_like(f)
    torch.cuda.synchronize()
    print(f"[bench] {label}: inputs ready: B={B} ws={ws.numel() / 2**30:.2f} GiB "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    # the library enqueues on torch's current stream: the events are recorded there
    stream = torch.cuda.current_stream()
    ev = []

    def step(timed):
        h = pmg.pmg_setup(desc, coords, ws, info)
        pmg.pmg_rhs(h, f, g, b)
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        pmg.pmg_solve(h, b, x, info)
        if timed:
            e1.record(stream)
            ev.append((e0, e1))
        pmg.pmg_lift(h, x, g, u)
        pmg.pmg_destroy(h)

    for i in range(warmup):
        step(False)
        torch.cuda.synchronize()
        print(f"[bench] {label}: warmup step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    nfo = pmg.info_to_numpy(info)
    ok = int(np.sum(nfo["status"] == 0))
    its = nfo["iterations"]
    solve_ms = [a.elapsed_time(bb) for a, bb in ev]
    solve_s = sum(solve_ms) / len(solve_ms) / 1e3
    ms_per_step = elapsed / steps * 1e3
    value = B * steps / elapsed
    print(f"[bench] {label}: timed {steps} steps: {ms_per_step:.1f} ms/step ({value:.1f} solves/s), "
          f"solve kernel {solve_s * 1e3:.1f} ms, ok {ok}/{B}, its min/med/max {its.min()}/"
          f"{int(np.median(its))}/{its.max()}, max relres {nfo['relres'].max():.2e}",
          file=sys.stderr, flush=True)
    # levels the library applies as dense matrices (named "Cc[l]" in the layout)
    coll = tuple(2 << int(name[3:-1]) for name, _, _ in pmg.pmg_workspace_layout(desc)
                 if name.startswith("Cc["))
    flops = sum(flops_per_solve(dim, p, gamma, 1, int(k), args.krylov, restart, coll, K)
                for k in its)
    xk = x[:keep].cpu().numpy() if keep else None
    return {"value": value, "ms_per_step": ms_per_step, "solve_s": solve_s, "its": its,
            "ok": ok, "flops": flops, "max_relres": float(nfo["relres"].max()),
            "probs": probs, "ps": ps, "x_keep": xk, "dim": dim, "p": p, "B": B,
            "gamma": gamma, "restriction": restriction, "prec": prec_name, "elements": K}


def roofline_of(r, prec_name):
    """Roofline of the dominant kernel (k_solve) from a run_batch result:
    algorithmic flops per launch / average launch duration (HIP events)."""
    achieved = r["flops"] / r["solve_s"] / 1e12
    peak = PEAK_FP32_TFLOPS if prec_name == "f32" else PEAK_FP64_TFLOPS
    tname = "float" if prec_name == "f32" else "double"
    kname = f"k_solve<{tname}, {r['p']}, {r['dim']}>"
    traffic, src = measured_traffic(kname, r["B"], r.get("elements", 1))
    # the solve's flops are mostly matrix-core contractions (operator and
    # transfers); MI355X's dense FP64 MFMA peak equals its FP64 vector peak.
    # Element hierarchies run their operator on the matrix cores where the
    # element degree is at least 16, else on the vector units.
    K = r.get("elements", 1)
    bound = "alu" if K > 1 and r["p"] // K < 16 else "mfma"
    return {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5), "traffic": traffic,
            "traffic_source": src if traffic is not None else None,
            "kernel": kname, "flops_per_launch": r["flops"],
            "avg_launch_ms": round(r["solve_s"] * 1e3, 3)}


def summary_of(r):
    import numpy as np
    return {"value": round(r["value"], 3), "unit": "solves/s", "ms_per_step": round(r["ms_per_step"], 3),
            "batch": r["B"], "gamma": r["gamma"], "restriction": r["restriction"],
            "iterations_median": int(np.median(r["its"])), "converged": r["ok"],
            "max_relres": r["max_relres"]}


def cr_words(n):
    return n if n <= 1 else n + cr_words(n // 2)


def components(args, probs, ps):
    """Rooflines of the two hot operations of the path, each launched alone
    through the library on the same batch (finest level): the sum-factorised
    operator (matrix cores; algorithmic flops) and the cyclic-reduction line
    solve (HBM; algorithmic bytes).  Durations come from HIP events on the
    launch stream around `reps` back-to-back launches."""
    import numpy as np
    import torch

    from paper_2504_10710_amd import pmg

    dev = torch.device("cuda:0")
    B, p, dim, reps = args.batch, args.p, 2, 10
    n1, n = p + 1, p - 1
    N = n1 ** dim
    coords = []
    for q in ps:
        xi = pmg.pmg_gll(q)[0]
        coords.append(torch.from_numpy(np.stack([pr.coords(xi) for pr in probs[:B]])).to(dev))
    out = {}
    stream = torch.cuda.current_stream()
    for prec_name in ("f64", "f32"):
        prec = pmg.PMG_F32 if prec_name == "f32" else pmg.PMG_F64
        tname = "float" if prec_name == "f32" else "double"
        esz = 4 if prec_name == "f32" else 8
        desc = pmg.make_desc(dim=dim, p_fine=p, batch=B, gamma=args.gamma, alpha=args.alpha,
                             smoother=pmg.PMG_SMOOTHER_FEM, inner_prec=prec)
        s = pmg.Solver(desc, coords)
        L = s.nlev - 1
        dt = torch.float32 if prec_name == "f32" else torch.float64
        gen = torch.Generator(device=dev).manual_seed(5)
        x = torch.randn(B, N, dtype=dt, device=dev, generator=gen)
        y = torch.empty_like(x)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps / 1e3

        t_apply = timed(lambda: pmg.pmg_apply(s.h, L, prec, x, y))
        fl = (8 * n1 + 7) * N * B          # four n1^3 contractions + pointwise fluxes
        peak = PEAK_FP32_TFLOPS if prec_name == "f32" else PEAK_FP64_TFLOPS
        out[f"k_apply<{tname}, {p}, 2>"] = {
            "bound": "mfma", "achieved": round(fl / t_apply / 1e12, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(fl / t_apply / 1e12 / peak, 4),
            "avg_ms": round(t_apply * 1e3, 4), "flops_per_problem": fl // B,
            "algorithmic_bytes_per_problem": (1 + 3 + 1) * N * esz}
        crw = cr_words(n)
        for d, nm in ((0, "x"), (1, "y")):
            # r in, z out, and the line data: lines solved by lane groups
            # (2-D, p <= 128) read their raw tridiagonal (3 words per unknown,
            # operators built on the fly), others the stored factors of every
            # CR level (3 CRW words)
            words = 3 * n if (d == 0 or dim == 2) and p <= 128 else 3 * crw
            nb = (2 * n ** dim + words * n ** (dim - 1)) * esz
            t = timed(lambda: pmg.pmg_line_solve(s.h, L, d, prec, x, y))
            gbs = nb * B / t / 1e9
            out[f"k_line_solve<{tname}, {p}, 2> {nm}-lines"] = {
                "bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                "frac": round(gbs / 8000.0, 4), "avg_ms": round(t * 1e3, 4),
                "algorithmic_bytes_per_problem": nb}
        del s
        torch.cuda.synchronize()
        print(f"[bench] components {prec_name}: " + ", ".join(
            f"{k} {v['achieved']} {v['unit']}" for k, v in out.items() if tname in k),
            file=sys.stderr, flush=True)
    return out


def sources_digest(root=ROOT):
    """SHA-256 (first 16 hex digits) of the kernel sources under csrc/."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(root, "paper_2504_10710_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, batch, elements=1, root=ROOT):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken on the current kernel sources at this batch size and element
    count (records without `elements` are one-element runs); else None."""
    import glob

    digest = sources_digest(root)
    for f in glob.glob(os.path.join(root, "profiles", "*.md")):
        rec = {}
        with open(f) as fh:
            for line in fh:
                if line.startswith("traffic-record:"):
                    for kv in line.split(":", 1)[1].split(";"):
                        if "=" in kv:
                            k, v = kv.split("=", 1)
                            rec[k.strip()] = v.strip()
        if rec.get("kernel") == kernel and rec.get("batch") == str(batch) and \
                rec.get("sources") == digest and rec.get("elements", "1") == str(elements):
            return float(rec["bytes_per_launch"]), os.path.basename(f)
    return None, digest


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; it has no multi-GPU "
                          "mode (independent problems shard by request across GPUs with no "
                          "collectives)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    # the oracle baseline runs first, on the host only, before the GPU is touched
    cpu, oracle_x = (cpu_baseline(args) if args.cpu_seconds > 0 else (None, []))

    import torch

    torch.cuda.set_device(0)
    B, p, dim = args.batch, args.p, 2
    keep = max(len(oracle_x), 1)
    r64 = run_batch(args, args.prec, keep=keep if args.elements == 1 else 0, tag="headline",
                    elements=args.elements)
    roofline = roofline_of(r64, args.prec)

    def oracle_err(r):
        if not oracle_x or r["x_keep"] is None:
            return None
        errs = [float(np.abs(r["x_keep"][i] - xo).max() / np.abs(xo).max())
                for i, xo in enumerate(oracle_x)]
        return {"max_rel_err_vs_fp64_oracle": max(errs), "problems": len(errs)}

    mixed = None
    if args.mixed and args.prec == "f64":
        r32 = run_batch(args, "f32", keep=keep if args.elements == 1 else 0, tag="mixed",
                        elements=args.elements)
        mixed = summary_of(r32)
        mixed.update({"dtype": "f32 cycle + f64 Krylov",
                      "speedup_vs_f64": round(r32["value"] / r64["value"], 3),
                      "roofline": roofline_of(r32, "f32"),
                      "error_vs_fp64_oracle": oracle_err(r32)})
    sweep = variants = None
    if args.sweep:
        sweep = {}
        for gam in (1, 2, 3, 7):
            r = r64 if gam == args.gamma else run_batch(args, "f64", gamma=gam, steps=2, warmup=0,
                                                        tag="sweep")
            sweep[f"gamma={gam}"] = summary_of(r)
        variants = {}
        for prec_name in ("f64", "f32"):
            r = run_batch(args, prec_name, gamma=1, restriction="transpose", steps=2, warmup=0,
                          tag="variant")
            v = summary_of(r)
            v["roofline"] = roofline_of(r, prec_name)
            variants[f"R=P^T gamma=1 {prec_name}"] = v
    legs = None
    if args.legs:
        legs = {}
        for (ldim, lp, lB, lgam, lrst) in ((3, 64, args.legs_batch3, args.gamma3, args.restriction3),
                                           (2, 256, 512, args.gamma, args.restriction)):
            for prec_name in ("f64", "f32"):
                r = run_batch(args, prec_name, dim=ldim, p=lp, B=lB, gamma=lgam, restriction=lrst,
                              steps=2, warmup=1, tag="leg")
                v = summary_of(r)
                v["interior_dofs"] = (lp - 1) ** ldim
                v["dof_per_s"] = round(r["value"] * (lp - 1) ** ldim, 1)
                v["roofline"] = roofline_of(r, prec_name)
                legs[f"{ldim}-D p={lp} {prec_name}"] = v
                torch.cuda.empty_cache()
        # multi-element hp-multigrid: 4 x 4 elements of degree 32 (the composite
        # grid of the p = 128 workload), FEM lines, exact solve at degree 8
        for prec_name in ("f64", "f32"):
            r = run_batch(args, prec_name, dim=2, p=128, B=args.batch, gamma=args.gamma,
                          restriction=args.restriction, steps=2, warmup=1, tag="leg", elements=4)
            v = summary_of(r)
            v["elements"] = "4x4, degree 32"
            v["interior_dofs"] = 127 ** 2
            v["dof_per_s"] = round(r["value"] * 127 ** 2, 1)
            v["roofline"] = roofline_of(r, prec_name)
            legs[f"2-D 4x4 elements p=32 {prec_name}"] = v
            torch.cuda.empty_cache()
    comps = components(args, r64["probs"], r64["ps"]) if args.components else None
    served = serve(args) if args.serve > 0 else None

    ndof = (p - 1) ** 2
    value = r64["value"]
    line = {
        "metric": "solves/s to 1e-10 rel. residual",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"2-D deformed square GLL Poisson, p={p}, gamma-cycle {p}->2"
                                if args.elements == 1 else
                                f"2-D deformed square, {args.elements}x{args.elements} GLL "
                                f"elements of degree {p // args.elements}, composite p={p}"),
                   "elements": args.elements,
                   "batch": B, "gamma": args.gamma, "m": 1, "alpha": args.alpha,
                   "smoother": args.smoother, "restriction": args.restriction,
                   "krylov": args.krylov, "rtol": args.rtol,
                   "inner_precision": args.prec, "interior_dofs": ndof,
                   "dof_per_s": round(value * ndof, 1),
                   "iterations_median": int(np.median(r64["its"])), "converged": r64["ok"],
                   "max_relres": r64["max_relres"],
                   "error_vs_fp64_oracle": oracle_err(r64)},
        "roofline": roofline,
        "kernels": comps,
        "cpu_baseline": cpu,
        "mixed_precision": mixed,
        "gamma_sweep": sweep,
        "variants": variants,
        "legs": legs,
        "serving": served,
    }
    print(json.dumps(line), flush=True)


# (dim, p, slots, inner precision, gamma, restriction).  A class with 1024
# slots can fill the chip by itself (256 CUs x 2 resident one-problem
# workgroups, twice over); 3-D p = 64 slots cost about 180 MB each, so that
# class holds 768.  2-D: the restriction by interpolation that reproduces
# Table 1, gamma per class the fastest on that shape.  3-D (the paper has no
# 3-D experiment to decide the restriction): R = P^T, gamma 1 (11 iterations
# at p = 64, where interpolation needs 69 at gamma 2 and 26 at gamma 4).
# 3-D p = 64 keeps the FP64 cycle: with the FP32 cycle and R = P^T about one
# problem in five of the served mix stagnates between 1e-8 and 1e-6.
SERVE_CLASSES = [
    (2, 16, 1024, "f32", 2, "interp"), (2, 32, 1024, "f32", 3, "interp"),
    (2, 64, 1024, "f32", 3, "interp"), (2, 128, 1024, "f32", 3, "interp"),
    (3, 16, 1024, "f32", 1, "transpose"), (3, 32, 1024, "f32", 1, "transpose"),
    (3, 64, 768, "f64", 1, "transpose"),
]


def _rst(name):
    from paper_2504_10710_amd import pmg
    return pmg.PMG_RESTRICT_INTERP if name == "interp" else pmg.PMG_RESTRICT_TRANSPOSE
SERVE_BUDGET_FRAC = 0.8     # admission budget: this share of the slot pools' bytes
SERVE_ITERS_PER_STEP = 16   # outer iterations of every running solve per server step
SERVE_ORACLE_SAMPLE = 4     # served results re-checked with the oracle's operator


def _request_arrays(item):
    """Host arrays of one request: per-level coordinates, f and g."""
    from paper_2504_10710_amd import inputs, pmg
    dim, p, prob = item
    ps = inputs.halving_degrees(p, 2)
    coords = [prob.coords(pmg.pmg_gll(q)[0]) for q in ps]
    X = coords[-1]
    return coords, prob.f(X), prob.g(X)


def serve(args):
    """Served stream: continuous batching of mixed 2-D/3-D requests through the
    library's server (FP32 cycle, FP64 Krylov, graph-replayed steps,
    byte-budget admission), every request its own seeded problem.  Pass 1
    submits every request at once (saturated throughput); pass 2 paces
    Poisson arrivals at serve_load x that throughput and reports per-request
    latency (arrival to retirement).  Baselines: the same requests solved
    the plain way, one batched pmg_solve per class, with the FP64 and with
    the FP32 cycle."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from paper_2504_10710_amd import inputs, pmg

    dev = torch.device("cuda:0")
    torch.cuda.empty_cache()         # the batch runs' workspaces go back first
    classes = []
    for dim, p, slots, prec, gam, rst in SERVE_CLASSES:
        classes.append(pmg.make_desc(dim=dim, p_fine=p, batch=slots, gamma=gam, alpha=0.16,
                                     smoother=pmg.PMG_SMOOTHER_FEM,
                                     inner_prec=pmg.PMG_F32 if prec == "f32" else pmg.PMG_F64,
                                     restart=30 if dim == 2 else 20, max_iter=400, rtol=1e-10,
                                     restriction=_rst(rst)))
    footprint = [pmg.pmg_pool_workspace_bytes(c) // c.batch for c in classes]
    budget = int(sum(f * c.batch for f, c in zip(footprint, classes)) * SERVE_BUDGET_FRAC)
    sdesc = pmg.make_server_desc(classes, iters_per_step=SERVE_ITERS_PER_STEP, budget_bytes=budget)
    stream = inputs.served_stream(args.serve, seed=7, amp_max=0.15)
    cls_of = {(d, p): i for i, (d, p, _, _, _, _) in enumerate(SERVE_CLASSES)}
    reqs = [cls_of[(d, p)] for d, p, _ in stream]
    n = len(reqs)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        host = list(ex.map(_request_arrays, stream))
    data = []
    for coords, f, g in host:
        data.append(([torch.from_numpy(c).to(dev).contiguous() for c in coords],
                      torch.from_numpy(f).to(dev), torch.from_numpy(g).to(dev)))
    del host
    torch.cuda.synchronize()
    print(f"[bench] serving: {n} requests, each its own problem, inputs ready "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    def run(arrivals):
        srv = pmg.pmg_server_create(sdesc, ws)
        outs, tickets, t_arr, t_done = [None] * n, [None] * n, np.zeros(n), np.zeros(n)
        nxt, done, its, worst = 0, 0, [], 0.0
        open_, req_of = set(), {}
        t0 = time.perf_counter()
        last_print = t0
        while done < n:
            if time.perf_counter() - last_print > 5.0:
                last_print = time.perf_counter()
                print(f"[bench] serving: {done}/{n} done, {nxt} arrived, "
                      f"{pmg.pmg_server_stats_get(srv)}", file=sys.stderr, flush=True)
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                coords, f, g = data[nxt]
                outs[nxt] = torch.empty_like(f)
                tickets[nxt] = pmg.pmg_server_submit(srv, reqs[nxt], coords, f, g, outs[nxt])
                req_of[tickets[nxt]] = nxt
                t_arr[nxt] = max(arrivals[nxt], 0.0)
                open_.add(nxt)
                nxt += 1
            st = pmg.pmg_server_stats_get(srv)
            if st["running"] == 0 and st["queued"] == 0:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)) if nxt < n else 0.0)
                continue
            if pmg.pmg_server_step(srv) == 0:
                continue
            now = time.perf_counter() - t0
            for t in pmg.pmg_server_drain(srv, n):
                i = req_of[int(t)]
                ok, info = pmg.pmg_server_poll(srv, int(t))
                assert ok and i in open_
                open_.discard(i)
                t_done[i] = now
                done += 1
                its.append(int(info["iterations"]))
                worst = float("inf") if info["status"] != 0 else max(worst, float(info["relres"]))
        makespan = time.perf_counter() - t0
        steps = pmg.pmg_server_stats_get(srv)["steps"]
        pmg.pmg_server_destroy(srv)
        lat = (t_done - t_arr) * 1e3
        last = {f"{d}d_p{p}": round(float(max((t_done[i] for i in range(n) if reqs[i] == c),
                                              default=0.0)), 4)
                for c, (d, p, _, _, _, _) in enumerate(SERVE_CLASSES)}
        return makespan, lat, steps, worst, its, last, outs

    def plain(prec):
        """The same requests solved the plain way: one one-shot batched
        pmg_solve per class over all of that class's requests (setup,
        lifting, solve, lift), classes back to back.  prec None: each class
        in the served class's own inner precision."""
        t0 = time.perf_counter()
        per_class = {}
        prec_all = prec
        for ci, (dim, p, _, cprec, gam, rst) in enumerate(SERVE_CLASSES):
            prec = prec_all if prec_all is not None else (
                pmg.PMG_F32 if cprec == "f32" else pmg.PMG_F64)
            idx = [i for i in range(n) if reqs[i] == ci]
            if not idx:
                continue
            tc = time.perf_counter()
            d = classes[ci]
            desc = pmg.make_desc(dim=dim, p_fine=p, batch=len(idx), gamma=gam, alpha=d.alpha,
                                 smoother=d.smoother, inner_prec=prec, restart=d.restart,
                                 max_iter=d.max_iter, rtol=d.rtol, restriction=_rst(rst))
            cs = [torch.stack([data[i][0][l] for i in idx]) for l in range(len(data[idx[0]][0]))]
            f = torch.stack([data[i][1] for i in idx])
            g = torch.stack([data[i][2] for i in idx])
            wsp = torch.empty(pmg.pmg_workspace_bytes(desc), dtype=torch.uint8, device=dev)
            info = torch.empty(len(idx) * pmg.INFO_BYTES, dtype=torch.uint8, device=dev)
            b = torch.empty_like(f)
            x = torch.empty_like(f)
            h = pmg.pmg_setup(desc, cs, wsp, info)
            pmg.pmg_rhs(h, f, g, b)
            pmg.pmg_solve(h, b, x, info)
            pmg.pmg_lift(h, x, g, b)
            torch.cuda.synchronize()
            nfo = pmg.info_to_numpy(info)
            bad = np.flatnonzero(nfo["status"] != 0)
            if len(bad):
                print(f"[bench] plain {dim}-D p={p} prec={prec}: {len(bad)} of {len(idx)} not "
                      f"converged: " + ", ".join(
                          f"req {idx[k]} status {nfo['status'][k]} its {nfo['iterations'][k]} "
                          f"relres {nfo['relres'][k]:.2e}" for k in bad[:8]),
                      file=sys.stderr, flush=True)
            failed[prec] = failed.get(prec, 0) + len(bad)
            pmg.pmg_destroy(h)
            del wsp, cs, f, g, b, x
            per_class[f"{dim}d_p{p}"] = round(time.perf_counter() - tc, 4)
        torch.cuda.empty_cache()
        return n / (time.perf_counter() - t0), per_class

    failed = {}
    plain(None)                      # warm-up (module load, graph-free path)
    failed.clear()
    plain64, plain64_cls = plain(pmg.PMG_F64)
    plain32, plain32_cls = plain(pmg.PMG_F32)
    plainc, plainc_cls = plain(None)
    print(f"[bench] served mix, plain batched per class: FP64 cycle {plain64:.1f}, FP32 cycle "
          f"{plain32:.1f}, served classes' precisions {plainc:.1f} solves/s (seconds per class "
          f"FP32: {plain32_cls})", file=sys.stderr, flush=True)
    ws = torch.empty(pmg.pmg_server_workspace_bytes(sdesc), dtype=torch.uint8, device=dev)
    mk, lat_sat, steps_sat, worst_sat, its, last_sat, outs_sat = run(np.zeros(n))
    print(f"[bench] served saturated: last completion per class (s): {last_sat}",
          file=sys.stderr, flush=True)
    # a sample of served results re-checked with the oracle's FP64 operator:
    # relative residual of w = u - v (interior) against the oracle's b
    check = oracle_check_served(stream, reqs, outs_sat) if args.cpu_seconds > 0 else None
    del outs_sat
    thr = n / mk
    rate = args.serve_load * thr
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    mk2, lat, steps, worst, _, _, _ = run(arrivals)
    mix = {f"{d}d_p{p}": int(sum(1 for c in reqs if SERVE_CLASSES[c][:2] == (d, p)))
           for d, p, _, _, _, _ in SERVE_CLASSES}
    print(f"[bench] served: saturated {thr:.1f} req/s, paced at {rate:.1f} req/s: "
          f"p50 {np.percentile(lat, 50):.1f} ms p99 {np.percentile(lat, 99):.1f} ms",
          file=sys.stderr, flush=True)
    return {"requests": n, "mix": mix, "distinct_problems": n,
            "inner_precision": {f"{d}d_p{p}": pr for d, p, _, pr, _, _ in SERVE_CLASSES},
            "gamma": {f"{d}d_p{p}": g for d, p, _, _, g, _ in SERVE_CLASSES},
            "restriction": {f"{d}d_p{p}": r for d, p, _, _, _, r in SERVE_CLASSES},
            "saturated_solves_per_s": round(thr, 2),
            "plain_fp64_batched_solves_per_s": round(plain64, 2),
            "plain_mixed_batched_solves_per_s": round(plain32, 2),
            "plain_mixed_seconds_per_class": plain32_cls,
            # the same per-class settings as served (FP32 cycle except 3-D p = 64):
            # what continuous batching adds over one batched solve per class
            "plain_served_settings_batched_solves_per_s": round(plainc, 2),
            "plain_served_settings_seconds_per_class": plainc_cls,
            "speedup_vs_plain_served_settings": round(thr / plainc, 3),
            "saturated_last_done_s": last_sat,
            "speedup_vs_plain_fp64": round(thr / plain64, 3),
            "speedup_vs_plain_mixed": round(thr / plain32, 3),
            "saturated_latency_ms": {"p50": round(float(np.percentile(lat_sat, 50)), 2),
                                     "p99": round(float(np.percentile(lat_sat, 99)), 2)},
            "paced_rate_per_s": round(rate, 2),
            "paced_solves_per_s": round(n / mk2, 2),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                           "p99": round(float(np.percentile(lat, 99)), 2)},
            "max_relres": worst, "iterations_median": int(np.median(its)),
            "plain_not_converged": {"fp64": failed.get(pmg.PMG_F64, 0),
                                    "mixed": failed.get(pmg.PMG_F32, 0),
                                    "served_settings": failed.get(None, 0)},
            "oracle_check": check,
            "budget_bytes": budget, "steps": int(steps), "iters_per_step": SERVE_ITERS_PER_STEP}


def oracle_check_served(stream, reqs, outs):
    """Relative FP64 residual, with the oracle's operator, of a sample of
    served solutions (the first requests of the small classes: 2-D p <= 64,
    3-D p = 16): w = u - v on the interior against the oracle's b = M f - A v."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2504_10710_amd import inputs

    worst, picked = 0.0, []
    for i, (dim, p, prob) in enumerate(stream):
        if len(picked) >= SERVE_ORACLE_SAMPLE:
            break
        if (dim == 2 and p > 64) or (dim == 3 and p > 16):
            continue
        ps = inputs.halving_degrees(p, 2)
        oc = [prob.coords(orc.gll(q)[0]) for q in ps]
        h = orc.Hier(dim, ps, oc, gamma=1, smoother=1, alpha=0.16)
        X = oc[-1]
        f, g = prob.f(X), prob.g(X)
        bo = h.rhs(f, g)
        u = outs[i].cpu().numpy()
        m1 = np.zeros(p + 1, dtype=bool)
        m1[1:-1] = True
        grids = np.meshgrid(*([m1] * dim), indexing="ij")
        interior = np.logical_and.reduce([gr.reshape(-1, order="F") for gr in grids])
        w = np.where(interior, u, 0.0)
        rr = float(np.linalg.norm(bo - h.apply(w)) / np.linalg.norm(bo))
        worst = max(worst, rr)
        picked.append({"request": i, "dim": dim, "p": p, "relres_oracle_operator": rr})
    return {"max_relres_oracle_operator": worst, "sample": picked}


def _oracle_solve(args, prob, ps):
    from oracle import oracle as orc
    oc = [prob.coords(orc.gll(q)[0]) for q in ps]
    h = orc.Hier(2, ps, oc, gamma=args.gamma, m=1, alpha=args.alpha,
                 smoother=1 if args.smoother == "fem" else 0,
                 restriction=orc.RESTRICT_INTERP if args.restriction == "interp" else orc.RESTRICT_TRANSPOSE)
    bo = h.rhs(prob.f(oc[-1]), prob.g(oc[-1]))
    x, st, it, _ = getattr(h, args.krylov)(bo, rtol=args.rtol, maxit=600)
    return x


def cpu_baseline(args):
    """The oracle (plain FP64 C) on a bounded sample of the headline workload:
    whole solves (setup + lifting + Krylov) of problems 0, 1, ... on one host
    core for about cpu_seconds, then distinct problems on every available core
    (a thread pool: the oracle's C calls release the interpreter lock) for
    about cpu_seconds.  Returns the record and the one-core solutions, which
    the GPU results are compared with."""
    import concurrent.futures as cf
    import threading

    from paper_2504_10710_amd import inputs

    ps = inputs.halving_degrees(args.p, 2)
    probs = make_problems(2, 64)
    t0 = time.perf_counter()
    xs = []
    while len(xs) < 1 or (time.perf_counter() - t0 < args.cpu_seconds and len(xs) < 8):
        xs.append(_oracle_solve(args, probs[len(xs)], ps))
    dt1 = time.perf_counter() - t0
    n1 = len(xs)
    print(f"[bench] oracle on one core: {n1} solves in {dt1:.1f} s", file=sys.stderr, flush=True)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    lock = threading.Lock()
    nxt = [n1]
    done = [0]
    t_end = time.perf_counter() + args.cpu_seconds

    def worker():
        while time.perf_counter() < t_end:
            with lock:
                i = nxt[0]
                nxt[0] += 1
            _oracle_solve(args, make_problems(2, 1, seed0=i)[0], ps)
            with lock:
                done[0] += 1

    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        for fut in [ex.submit(worker) for _ in range(cores)]:
            fut.result()
    dtn = time.perf_counter() - t1
    print(f"[bench] oracle on {cores} cores: {done[0]} solves in {dtn:.1f} s", file=sys.stderr,
          flush=True)
    rec = {"value": round(n1 / dt1, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": f"{n1} whole solves of the headline workload (problems 0..{n1 - 1}), "
                     f"{dt1:.1f} s on one host core",
           "all_cores": {"value": round(done[0] / dtn, 4), "unit": "solves/s", "cores": cores,
                         "sample": f"{done[0]} whole solves of distinct problems, {dtn:.1f} s "
                                   f"on {cores} threads"}}
    return rec, xs


if __name__ == "__main__":
    main()
