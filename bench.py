#!/usr/bin/env python
"""Seconds per geometry for SCCSD(E) energies + gradients + couplings on one
MI355X, with the FP64 MFMA contraction roofline and the CPU oracle timed on a
bounded sample.  Prints one JSON line.

Workload (default o10v90): synthetic Cholesky-factored Hamiltonian with
o = 10, v = 90, N_J = 300, 3 excited states, 36 coordinates, 3 pairwise
couplings.  One step is one geometry x of the trajectory family
H(x) = H0 + sum_k x_k H_k (x_k ~ N(0, 0.05^2), a new x every step, H(x)
already on the device): RHF in the fixed basis and MO transformation on the
device, SCCSD(E) ground + excited states from a cold start, gradients of all
3 states and 3 couplings over all coordinates.

The warm-up and timed loops stop early at their wall budgets (--warmup-budget,
--budget, seconds): the JSON line reports the steps actually run.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the counter runs recorded in
    profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a
    plain copy of known size); None unless they were taken over this
    workload with the kernel source as it is now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, "paper_2403_01007_amd", "csrc", "exec.hip"), "rb").read()
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def oracle_baseline(S, workload, iterations=25):
    """The FP64 CPU oracle on the host cores, on a bounded sample of this
    workload: `iterations` steps of its own CCSD ground-state iteration (the
    residual with full N^4 integrals plus its DIIS step) at x = 0, scaled to
    one geometry by the oracle's whole-geometry time in units of the same
    step, from its complete run of a three-state system (three gradients,
    three couplings; tests/golden/<name>.json, written by scripts that call
    only the oracle)."""
    import numpy as np
    import torch
    from oracle import cc
    from oracle import scc as oscc
    threads = len(os.sched_getaffinity(0))
    torch.set_num_threads(threads)
    ref, ref_name = {}, None
    for name in ("o6v26", "o4v12s3"):
        ref_path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
        if os.path.exists(ref_path):
            ref = json.load(open(ref_path)).get("oracle_timing", {})
            if "ground_iteration_seconds" in ref:
                ref_name = name
                break
    if ref_name is None:
        return None
    h, L = S.at(np.zeros(S.ncoord))
    ht = torch.as_tensor(h)
    gt = cc.chol_to_g(torch.as_tensor(L))
    eps = np.diag(cc.fock(ht, gt, S.o).numpy()).copy()

    def steps(n):
        c0 = time.perf_counter()
        try:
            oscc.solve_ground(ht, gt, S.o, eps, tol=0.0, maxiter=n)
        except RuntimeError:
            pass  # tol = 0: the iteration always stops at its step limit
        return time.perf_counter() - c0

    # a two-step probe sizes the sample to about 20 s of CPU work
    iterations = int(min(iterations, max(2, round(20.0 / max(steps(2) / 2, 1e-3)))))
    t_step = steps(iterations) / iterations
    ratio = (ref["solve_seconds"] + ref["targets_seconds"]) / ref["ground_iteration_seconds"]
    return {"value": t_step * ratio, "unit": "s/geometry", "cores": threads, "kind": "oracle",
            "sample": (f"{iterations} steps of the oracle's CCSD ground-state iteration at {workload} "
                       f"({t_step:.2f} s per step, torch CPU FP64 with N^4 integrals) times {ratio:.0f}, the "
                       f"oracle's whole-geometry time in units of that step in its complete {ref_name} run "
                       f"(energies, 3 gradients, 3 couplings; tests/golden/{ref_name}.json, {ref['threads']} threads)")}


def calibration_copy(dev):
    """A plain device copy of known size (512 MiB read, 512 MiB written)."""
    import torch
    cal_src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst


def learned_main(args):
    """Learned initial guesses on the trajectory family H(x) = H0 + sum_k x_k H_k:
    solve the training geometries (energies, gradients and couplings of every
    target, collecting amplitudes, right vectors, zeta and the multipliers of
    every target), fit PCA bases of each family on the device, train the
    perceptron on the device, then solve held-out geometries from the plain
    start and from the predicted start (every prediction judged by the
    solvers' residuals, with the plain start as fallback)."""
    import numpy as np
    import torch
    from paper_2403_01007_amd import Context
    from paper_2403_01007_amd.binding import FIELD_R, FIELD_T, Mlp, SccError, pca_expand, pca_fit
    from synth_inputs import family_geometries, make_system

    S = make_system(args.learned_workload)
    dev = torch.device("cuda:0")
    mk = lambda tol, verbose=False: Context(S.o, S.v, S.nj, S.nstates, tol=tol, tol_overlap=0.1 * tol,
                                            verbose=verbose)
    ns, npair = S.nstates, S.nstates * (S.nstates - 1) // 2
    states, pairs = list(range(ns)), list(S.nacs)
    nt = len(states) + len(pairs)
    dh = torch.as_tensor(S.dh, device=dev)
    dL = torch.as_tensor(S.dL, device=dev)

    def solve(ctx, x, guess=None, keep=False):
        h, L = S.at(x)
        ctx.set_hamiltonian_fixed_basis(torch.as_tensor(h, device=dev), torch.as_tensor(L, device=dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it_g, fb_g = 0, 0
        if guess is not None:
            _, info = ctx.ground(guess["t"])
            it_g, fb_g = info.iterations, info.fallback_used
        E, z, info = ctx.excited(None if guess is None else guess["r"])
        it_e, fb_e = info.iterations + it_g, info.fallback_used
        torch.cuda.synchronize()
        t_exc = time.perf_counter() - t0
        res = ctx.gradients_and_couplings(states, pairs, dh, dL, guess=None if guess is None else guess["m"],
                                          multipliers=keep)
        g, d, info = res[:3]
        torch.cuda.synchronize()
        out = dict(E=np.asarray(E), zeta=np.asarray(z), g=g, d=d, t_exc=t_exc, t_all=time.perf_counter() - t0,
                   it_exc=it_e, it_mult=info.iterations, fallback=fb_g or fb_e or info.fallback_used,
                   fb=(fb_g, fb_e, info.fallback_used))
        if keep:
            out["M"] = res[3]
        return out

    # training geometries at the training tolerance; those that do not
    # converge from the plain start are left out (and counted)
    Xtr = family_geometries(S.ncoord, range(10000, 10000 + args.ntrain))
    Xte = family_geometries(S.ncoord, range(20000, 20000 + args.nheld))
    nst = 1 + S.o * S.v * (1 + S.o * S.v)
    ctx = mk(args.train_tol)
    nm = ctx.multiplier_length()
    Tm = torch.empty((args.ntrain, nst - 1), dtype=torch.float64, device=dev)
    Rm = torch.empty((args.ntrain, ns * nst), dtype=torch.float64, device=dev)
    Mm = torch.empty((args.ntrain, nt * nm), dtype=torch.float64, device=dev)
    Zm = np.zeros((args.ntrain, npair))
    t0 = time.perf_counter()
    used, skipped_train = [], 0
    for i, x in enumerate(Xtr):
        try:
            r = solve(ctx, x, keep=True)
        except SccError as e:
            skipped_train += 1
            print(f"[learned: training geometry {i} skipped: {e}]", file=sys.stderr, flush=True)
            ctx.close()
            torch.cuda.empty_cache()
            ctx = mk(args.train_tol)
            continue
        q = len(used)
        Tm[q] = ctx.get(FIELD_T)
        for k in range(ns):
            Rm[q, k * nst:(k + 1) * nst] = ctx.get(FIELD_R, k)
        Mm[q] = r["M"].reshape(-1)
        Zm[q] = r["zeta"]
        used.append(i)
        print(f"[learned: training geometry {i} done ({r['t_all']:.1f} s)]", file=sys.stderr, flush=True)
    ctx.close()
    torch.cuda.empty_cache()  # the next contexts need the whole workspace block back
    ntr = len(used)
    Xtr, Tm, Rm, Mm, Zm = Xtr[used], Tm[:ntr], Rm[:ntr], Mm[:ntr], Zm[:ntr]
    t_data = time.perf_counter() - t0
    kt = min(64, ntr - 1)
    mt, Ut, Ct, _ = pca_fit(Tm, kt)
    mr, Ur, Cr, _ = pca_fit(Rm, kt)
    mm, Um, Cm, _ = pca_fit(Mm, kt)
    del Tm, Rm, Mm
    Y = np.concatenate([Ct.cpu().numpy(), Cr.cpu().numpy(), Cm.cpu().numpy(), Zm], axis=1)
    # the network learns standardised outputs (every PCA coefficient and zeta
    # with zero mean and unit spread over the training set)
    ymu, ysd = Y.mean(axis=0), Y.std(axis=0) + 1e-12
    Y = (Y - ymu) / ysd
    ymu_d, ysd_d = torch.as_tensor(ymu, device=dev), torch.as_tensor(ysd, device=dev)
    nout = Y.shape[1]
    rng = np.random.Generator(np.random.PCG64(4242))
    nh = 256
    sizes = [(nh, S.ncoord), (nh,), (nh, nh), (nh,), (nout, nh), (nout,)]
    p0 = np.concatenate([rng.normal(0, 1.0 / np.sqrt(sh[1]), size=sh).ravel() if len(sh) == 2 else np.zeros(sh)
                         for sh in sizes])
    net = Mlp(S.ncoord, nh, nout, p0)
    batch = min(64, ntr)
    order = np.stack([rng.permutation(ntr)[:batch] for _ in range(args.train_steps)])
    t1 = time.perf_counter()
    losses = net.train(Xtr, Y, order, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    print(f"[learned: {ntr} training geometries in {t_data:.1f} s; trained {args.train_steps} steps in "
          f"{t_train:.2f} s, loss {losses[0]:.3e} -> {losses[-20:].mean():.3e}]", file=sys.stderr, flush=True)
    # held-out geometries at the benchmark tolerance: plain start on a fresh
    # context each, learned start on one context along the held-out sequence
    plain, learned = [], []
    lctx = mk(1e-10, args.verbose)
    failed = 0
    for i, x in enumerate(Xte):
        pctx = mk(1e-10)
        try:
            rp = solve(pctx, x)
        except SccError as e:
            print(f"[learned: held-out geometry {i} skipped (plain start): {e}]", file=sys.stderr, flush=True)
            pctx.close()
            torch.cuda.empty_cache()
            continue
        pctx.close()
        torch.cuda.empty_cache()
        c0 = time.perf_counter()
        yp = net.forward(x[None, :]).to(torch.float64) * ysd_d + ymu_d
        guess = {"t": pca_expand(mt, Ut, yp[:, :kt])[0],
                 "r": torch.cat([pca_expand(mr, Ur, yp[:, kt:2 * kt])[0], yp[0, 3 * kt:]]),
                 "m": pca_expand(mm, Um, yp[:, 2 * kt:3 * kt])[0].reshape(nt, nm)}
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - c0
        try:
            rl = solve(lctx, x, guess)
        except SccError as e:
            failed += 1
            print(f"[learned: held-out geometry {i} failed from the learned start: {e}]", file=sys.stderr, flush=True)
            lctx.close()
            torch.cuda.empty_cache()
            lctx = mk(1e-10, args.verbose)
            continue
        rl["t_exc"] += t_pred
        rl["t_all"] += t_pred
        plain.append(rp)
        learned.append(rl)
        print(f"[learned: held-out {i}: plain {rp['t_all']:.1f} s ({rp['it_exc']}+{rp['it_mult']} it), learned "
              f"{rl['t_all']:.1f} s ({rl['it_exc']}+{rl['it_mult']} it), fallbacks ground/excited/multipliers "
              f"{rl['fb']}]", file=sys.stderr, flush=True)
    mean = lambda rs, key: float(np.mean([r[key] for r in rs]))
    diff = lambda key: max(float(np.abs(np.asarray(a[key]) - np.asarray(b[key])).max()) for a, b in zip(plain, learned))
    line = {
        "metric": "s/geometry (energies+gradients+NACs), MFMA TFLOP/s; mixed+learned vs FP64",
        "value": mean(learned, "t_all"), "unit": "s/geometry", "n_gpus": 1, "steps": len(learned), "warmup": 0,
        "ms_per_step": 1e3 * mean(learned, "t_all"), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.learned_workload, "guess": "learned", "ntrain": ntr,
                   "train_tol": args.train_tol, "nheld": len(learned), "pca": kt, "mlp": [S.ncoord, nh, nh, nout],
                   "skipped_training": skipped_train, "failed_learned": failed},
        "learned": {"plain_s_per_geometry": mean(plain, "t_all"), "learned_s_per_geometry": mean(learned, "t_all"),
                    "speedup": mean(plain, "t_all") / mean(learned, "t_all"),
                    "plain_excited_s": mean(plain, "t_exc"), "learned_excited_s": mean(learned, "t_exc"),
                    "plain_iterations_excited": mean(plain, "it_exc"),
                    "learned_iterations_excited": mean(learned, "it_exc"),
                    "plain_iterations_multipliers": mean(plain, "it_mult"),
                    "learned_iterations_multipliers": mean(learned, "it_mult"),
                    "fallbacks": int(sum(r["fallback"] for r in learned)),
                    "fallbacks_ground_excited_multipliers": [int(sum(r["fb"][q] for r in learned)) for q in range(3)],
                    "max_abs_diff_energy": diff("E"), "max_abs_diff_gradient": diff("g"),
                    "max_abs_diff_coupling": diff("d"),
                    "training_data_s": t_data, "training_s": t_train, "final_loss": float(losses[-20:].mean())},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget", type=float, default=120.0,
                    help="wall budget (s) of the timed loop: no step starts that would end past it (at least one "
                         "step runs)")
    ap.add_argument("--warmup-budget", type=float, default=60.0,
                    help="wall budget (s) of the warm-up loop (at least one warm-up step runs when --warmup > 0)")
    ap.add_argument("--workload", default="o10v90")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="fp32: FP32 products in the dense contractions, then FP64 refinement")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="with --precision fp32: also solve one geometry in FP64 (untimed) and report the "
                         "largest differences and the FP64 time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one (no HIP graphs)")
    ap.add_argument("--no-roofline", action="store_true", help="no per-GEMM event timing in the timed region")
    ap.add_argument("--all-gemm-events", action="store_true",
                    help="events around every GEMM kernel's launches in the timed region (default: the "
                         "multi-product kernel's only)")
    ap.add_argument("--one-target-at-a-time", action="store_true",
                    help="solve the multiplier equations of each gradient / coupling separately")
    ap.add_argument("--learned", action="store_true",
                    help="learned initial guesses: train on the trajectory family, time held-out geometries")
    ap.add_argument("--learned-workload", default="o4v12x36")
    ap.add_argument("--ntrain", type=int, default=200)
    ap.add_argument("--nheld", type=int, default=20)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--train-tol", type=float, default=1e-8,
                    help="residual tolerance of the training solves (the held-out solves use 1e-10)")
    ap.add_argument("--calibration-only", action="store_true",
                    help="only the 512 MiB device copy that scales HBM traffic counters, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (there is no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.learned:
        learned_main(args)
        return
    import numpy as np
    import torch
    if args.calibration_only:
        calibration_copy(torch.device("cuda:0"))
        return
    from paper_2403_01007_amd import Context
    from paper_2403_01007_amd.binding import GEMM_KERNEL_NAMES
    from synth_inputs import family_geometries, make_system

    S = make_system(args.workload)
    h, L = S.at(np.zeros(S.ncoord))
    dev = torch.device("cuda:0")
    # one geometry of the trajectory family per step, H(x) formed and moved to
    # the device before the timed region (held-out seeds 20000+)
    nstep_max = args.warmup + args.steps
    geoms = family_geometries(S.ncoord, range(20000, 20000 + nstep_max))
    HX = []
    for x in geoms:
        hx, Lx = S.at(x)
        HX.append((torch.as_tensor(hx, device=dev), torch.as_tensor(Lx, device=dev)))
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-10, tol_overlap=1e-11, verbose=args.verbose,
                  precision=args.precision, eager=args.eager)
    h_d = torch.as_tensor(h, device=dev)
    L_d = torch.as_tensor(L, device=dev)
    dh = torch.as_tensor(S.dh, device=dev)
    dL = torch.as_tensor(S.dL, device=dev)
    flops = [0.0]

    def phase(name, info):
        flops[0] += info.flops_mfma
        if args.verbose:
            print(f"[phase {name}: {info.seconds:.2f} s, {info.iterations} iterations, "
                  f"{info.flops_mfma / 1e12:.2f} TFLOP]", file=sys.stderr, flush=True)

    def step(i, ctx=ctx):
        hx, Lx = HX[i]
        _, info = ctx.set_hamiltonian_fixed_basis(hx, Lx)
        phase("rhf", info)
        E, zeta, info = ctx.excited()
        phase("excited", info)
        out = {"E": E, "zeta": zeta}
        if args.one_target_at_a_time:
            for n in range(S.nstates):
                g, info = ctx.gradient(n, dh, dL)
                phase(f"gradient {n}", info)
                out[f"g{n}"] = g
            for (m, n) in S.nacs:
                d, info = ctx.nac(m, n, dh, dL)
                phase(f"coupling {m},{n}", info)
                out[f"d{m}{n}"] = d
            return out
        g, d, info = ctx.gradients_and_couplings(list(range(S.nstates)), list(S.nacs), dh, dL)
        phase(f"{S.nstates} gradients + {len(S.nacs)} couplings", info)
        for n in range(S.nstates):
            out[f"g{n}"] = g[n]
        for i, (m, n) in enumerate(S.nacs):
            out[f"d{m}{n}"] = d[i]
        return out

    reference = None
    if args.precision == "fp32" and args.compare_fp64:
        ref_ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-10, tol_overlap=1e-11, verbose=args.verbose)
        r0 = time.perf_counter()
        reference = step(args.warmup, ref_ctx)
        torch.cuda.synchronize()
        reference["seconds"] = time.perf_counter() - r0
        ref_ctx.close()
        del ref_ctx
        print(f"[fp64 reference geometry done: {reference['seconds']:.1f} s]", file=sys.stderr, flush=True)
    # a plain device copy of known size (512 MiB) outside the timed region:
    # the reference that scales HBM traffic counters taken over this command
    calibration_copy(dev)
    # load the kernels and touch every code path once outside the timed region
    ctx.set_hamiltonian(h_d, L_d)
    ctx.eval_residual(np.zeros(S.o * S.v * (1 + S.o * S.v)))
    # warm-up: no step starts that would end past the warm-up budget
    warm_run = 0
    w0 = time.perf_counter()
    for i in range(args.warmup):
        s0 = time.perf_counter()
        step(i)
        torch.cuda.synchronize()
        warm_run += 1
        last = time.perf_counter() - s0
        print(f"[warmup step {i} done: {last:.1f} s]", file=sys.stderr, flush=True)
        if time.perf_counter() - w0 + last > args.warmup_budget:
            break
    flops[0] = 0.0
    kernels = range(len(GEMM_KERNEL_NAMES))
    # events on the multi-product GEMM launches only (the dominant kernel by
    # the kernel trace), unless every GEMM kernel is asked for
    if not args.all_gemm_events:
        ctx.profile_kernels([GEMM_KERNEL_NAMES.index("gemm_f64_multi_kernel"),
                             GEMM_KERNEL_NAMES.index("gemm_f32acc_multi_kernel")])
    before = [ctx.profile(not args.no_roofline, q) for q in kernels]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_run = 0
    for k in range(args.steps):
        s0 = time.perf_counter()
        res = step(args.warmup + k)
        torch.cuda.synchronize()
        steps_run += 1
        last = time.perf_counter() - s0
        print(f"[timed step {k} done: {last:.1f} s]", file=sys.stderr, flush=True)
        if time.perf_counter() - t0 + last > args.budget:
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    after = [ctx.profile(False, q) for q in kernels]
    s_per_geom = elapsed / steps_run
    # per GEMM kernel over the timed steps: seconds, flops, launches; the
    # roofline is that of the kernel with the most time
    per_kernel = {GEMM_KERNEL_NAMES[q]: ((after[q][0] - before[q][0]) / 1e3, after[q][1] - before[q][1],
                                         after[q][2] - before[q][2], after[q][3] - before[q][3]) for q in kernels}
    top = max(per_kernel, key=lambda k: per_kernel[k][0])
    gemm_s, gemm_fl, gemm_n, gemm_by = per_kernel[top]
    achieved = gemm_fl / gemm_s / 1e12 if gemm_s > 0 else 0.0
    peak = PEAK_FP64_MFMA if "f64" in top else PEAK_FP32_MFMA

    # flops of one residual evaluation: the work of a geometry in units of
    # the ground-state residual ("transformations" per geometry)
    nov = S.o * S.v
    t_zero = np.zeros(nov + nov * nov)
    ctx.profile_kernels(kernels)
    a_fl = sum(ctx.profile(True, q)[1] for q in kernels)
    ctx.eval_residual(t_zero)
    b_fl = sum(ctx.profile(True, q)[1] for q in kernels)
    ctx.profile(False)
    res_flops = b_fl - a_fl

    traffic = stored_traffic(top, args.workload)
    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = oracle_baseline(S, args.workload)
        except Exception as e:  # the GPU figures stand without it
            print(f"[cpu baseline failed: {e}]", file=sys.stderr, flush=True)

    line = {
        "metric": "s/geometry (energies+gradients+NACs), MFMA TFLOP/s; mixed+learned vs FP64",
        "value": s_per_geom, "unit": "s/geometry", "n_gpus": 1, "steps": steps_run, "warmup": warm_run,
        "steps_requested": args.steps, "warmup_requested": args.warmup,
        "ms_per_step": 1e3 * s_per_geom, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-products+f64", "data": "synthetic",
        "config": {"workload": args.workload, "o": S.o, "v": S.v, "nchol": S.nj, "nstates": S.nstates,
                   "ncoord": S.ncoord, "nacs": len(S.nacs), "precision": args.precision, "guess": "mp2/unit",
                   "generator": S.reading},
        "tflops_contractions": (flops[0] / steps_run) / s_per_geom / 1e12,
        "transformations_per_geometry": (flops[0] / steps_run) / res_flops if res_flops > 0 else None,
        "roofline": {"bound": "mfma", "kernel": top, "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic, "launches": gemm_n, "kernel_seconds": gemm_s,
                     "algorithmic_bytes_per_launch": gemm_by / gemm_n if gemm_n else None,
                     "gemm_kernels": {k: {"seconds": v[0], "launches": v[2],
                                          "tflops": v[1] / v[0] / 1e12 if v[0] > 0 else 0.0}
                                      for k, v in per_kernel.items() if v[2] > 0}},
        "cpu_baseline": cpu,
        "energies": [float(x) for x in res["E"]],
    }
    if reference is not None:
        def maxdiff(prefix):
            keys = [k for k in res if k.startswith(prefix)]
            return max(float(np.abs(np.asarray(res[k]) - np.asarray(reference[k])).max()) for k in keys)
        line["vs_fp64"] = {"fp64_seconds": reference["seconds"], "speedup": reference["seconds"] / s_per_geom,
                           "max_abs_diff_energy": float(np.abs(res["E"] - reference["E"]).max()),
                           "max_abs_diff_gradient": maxdiff("g"), "max_abs_diff_coupling": maxdiff("d")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
