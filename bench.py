#!/usr/bin/env python3
"""Walker-step throughput of the phaseless-AFQMC hot path on one MI355X.

One walker-step = propagation (overlap/LU, force bias, V_HS, B1 T6(sqrt(dt) V_HS)
B1, weight update) + local energy (one-body, Coulomb, exchange, estimator), with
re-orthogonalisation every 5th step, for every walker of the headline workload
(M=400 orbitals, 40+40 electrons, 1600 Cholesky vectors, 256 walkers, dt=0.005;
seeded synthetic Hamiltonian, trial and fields, resident in HBM before timing).

By default the FP64 path and the precision form (exchange and force bias as
the trial split: the trial's part of the Green's function exact, the walker's
departure from it in one FP16 product with FP32 accumulation; everything else
FP64) are both timed, with the split-BF16 form (two bfloat16 terms per operand,
three products) beside them; the JSON line reports the precision form's
walker-steps/s, its speed-up over FP64, and its per-walker energy error against
the FP64 path on identical walker states (the bar is 0.1 mHa).  The roofline object is the dominant kernel (exchange) of the reported
path, timed by the library's HIP-event phase timers inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s (propagate+energy) at M=400,N=40; speed-up vs FP64 at 0.1 mHa"
METRIC_FREE = "free-projection walker-steps/s (propagate+energy) at M=400,N=40; speed-up vs FP64"
# dense MI355X peaks per arithmetic type (TFLOP/s)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x2": 2500.0, "fp16t": 2500.0, "bf16t": 2500.0}
PRECISION_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x2": 3, "fp16t": 4, "bf16t": 5}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6, "bf16x2": 3, "fp16t": 1, "bf16t": 1}


KERNEL_NAME = {"fp64": "k_exchange_mfma", "fp32": "k_exchange_f32", "bf16x3": "k_exchange_bf16<40,3>",
               "bf16x2": "k_exchange_bf16<40,2>", "fp16t": "k_exchange_bf16<40,1,_Float16>",
               "bf16t": "k_exchange_bf16<40,1,__bf16>"}
KERNEL_SOURCE = {"k_exchange_mfma": "k_exchange.hip", "k_exchange_f32": "k_exchange_lp.hip",
                 "k_exchange_bf16<40,3>": "k_exchange_lp.hip", "k_exchange_bf16<40,2>": "k_exchange_lp.hip",
                 "k_exchange_bf16<40,1,_Float16>": "k_exchange_lp.hip", "k_exchange_bf16<40,1,__bf16>": "k_exchange_lp.hip"}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "exchange_hbm_traffic.md")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    profile, or None when there is none for this workload or the kernel's
    source has changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2406_16238_amd", "csrc", KERNEL_SOURCE[kernel])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return None
    for line in lines:
        # machine-readable rows: "traffic <kernel> <workload> <bytes per launch> <source sha256[:16]>"
        f = line.strip().strip("`").split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[2] == workload:
            return float(f[3]) if f[4] == digest else None
    return None


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "medium", "small", "batching", "cv", "stat"],
                    help="batching: the sixteen-system set (aggregate walker-steps/s of separate contexts run "
                         "one after another, of one set context over internal streams, and of that context "
                         "replaying a hipGraph); cv: the learned control variate at the headline shape "
                         "(training on the path's own trajectory, then full exchange vs the 1/8 subset)")
    ap.add_argument("--precision", default="fp16t", choices=["fp64", "fp32", "bf16x3", "bf16x2", "fp16t", "bf16t"],
                    help="path reported in the JSON line (the FP64 path is timed too, for the speed-up)")
    ap.add_argument("--prop-precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the propagation (V_HS planes and Taylor terms) of the reported path")
    ap.add_argument("--projection", default="phaseless", choices=["phaseless", "free"],
                    help="phaseless AFQMC (the headline) or free projection (same kernels, bare fields, "
                         "complex amplitudes)")
    ap.add_argument("--api", default="step", choices=["step", "separate"],
                    help="step: afqmc_step (one overlap/LU and one force bias per step); separate: "
                         "afqmc_propagate + afqmc_reorthogonalize + afqmc_local_energy")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-legs", action="store_true",
                    help="headline only: skip the other workloads' legs (medium FP64, reblocked energies of every "
                         "form, the sixteen-system set, the control variate at headline and benzene scale)")
    ap.add_argument("--cv-train-steps", type=int, default=60, help="cv: trajectory steps whose walkers train the network")
    ap.add_argument("--cv-epochs", type=int, default=30, help="cv: training passes")
    ap.add_argument("--cv-draws", type=int, default=60, help="cv: subset draws at fixed walkers")
    ap.add_argument("--cv-system", default="headline", choices=["headline", "benzene"],
                    help="cv: the headline shape, or M=1512, N=42+42, 6000 Cholesky vectors, 64 walkers with the "
                         "Cholesky tensor drawn on the device")
    ap.add_argument("--no-prop32-leg", action="store_true",
                    help="skip timing the reported form with FP32 propagation as well")
    ap.add_argument("--repeats", type=int, default=4,
                    help="further timed blocks of --steps steps after the reported one (their walker-steps/s and "
                         "the median of all blocks are reported beside value)")
    ap.add_argument("--cpu-walkers", type=int, default=32, help="walkers in the CPU oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=6, help="steps in the CPU oracle sample")
    ap.add_argument("--phases", action="store_true", help="print the per-phase tables to stderr")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the run, copy a device buffer of this many MiB (a plain copy kernel of known "
                         "size, for scaling the HBM byte counters of a profile)")
    return ap.parse_args(argv)


def exchange_flops(M, na, nb, G, W):
    """Algorithmic flops of one exchange launch pair (both spins): T = Ltilde Theta
    (real x complex, 4 flops per (i, j, q)) and the trace sum_ij T_ij T_ji."""
    n2 = na * na + nb * nb
    return float(W) * (4.0 * n2 * M * G + 8.0 * n2 * G)


def step_flops(M, na, nb, G, free=False):
    """Algorithmic flops of one walker-step (both spins, real L and trial,
    complex walkers): exchange + trace + V_HS + Taylor(6) + B1 (twice) + force
    bias + overlaps and solves.  Free projection: real fields, so V_HS is a
    real combination of the L^g and each Taylor term a real-by-complex product."""
    n2 = na * na + nb * nb
    nt = na + nb
    f = 0.5 if free else 1.0
    return (4.0 * n2 * M * G + 8.0 * n2 * G + f * 4.0 * G * M * M + f * 6 * 8.0 * M * M * nt
            + 2 * 4.0 * M * M * nt + 4.0 * G * M * nt + 2 * 16.0 * M * n2)


def exchange_roofline(prec, phases, M, s, G, W, workload):
    """Roofline object of the exchange kernel (the step's dominant one): the
    algorithmic flops of one launch (one spin block of every walker) over its
    average launch time from the library's HIP-event phase timers."""
    ex_ms, ex_n = phases["exchange"]
    blocks = [n for n in (s.nalpha, s.nbeta) if n > 0]
    ex_flops = exchange_flops(M, s.nalpha, s.nbeta, G, W) / len(blocks)
    avg_ms = ex_ms / max(ex_n, 1)
    achieved = ex_flops / (avg_ms * 1e-3) / 1e12 if ex_n else 0.0
    kernel = KERNEL_NAME[prec]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[prec], 4), "traffic": measured_traffic(kernel, workload),
            "kernel": f"{kernel} (one spin block of {W} walkers per launch)", "avg_launch_ms": round(avg_ms, 4),
            "flops_per_launch": ex_flops, "executed_tflops": round(achieved * PRODUCTS[prec], 3)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, n_walkers, n_steps, free=False):
    """The CPU oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    import afqmc_inputs as gi
    from oracle import afqmc_oracle as O
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        blas_threads = int(blas[0]["num_threads"]) if blas else 1
    except Exception:
        blas_threads = None
    s = spec.system
    h1, chol, ecore, trial = gi.make_system(s)
    ham = O.build(h1, chol, ecore, trial, s.nalpha, s.nbeta, spec.dt)
    phis = gi.initial_walkers(trial, n_walkers)
    fields = gi.FieldStream(spec.field_seed, n_walkers, s.nchol)
    w = np.ones(n_walkers)
    logo = O.initial_logo(ham, phis)
    amp = O.initial_amplitudes(logo)
    t0 = time.perf_counter()
    for k in range(1, n_steps + 1):
        if free:
            phis, logo, amp, _ = O.free_propagate(ham, phis, logo, amp, fields.next())
        else:
            phis, w, logo, _ = O.propagate(ham, phis, w, logo, fields.next())
        if k % spec.reortho_every == 0:
            phis, logo = O.reorthogonalize(ham, phis, logo)
        O.local_energies(ham, phis)
    dt = time.perf_counter() - t0
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            p1 = gi.initial_walkers(trial, 8)
            w1, l1 = np.ones(8), O.initial_logo(ham, p1)
            a1 = O.initial_amplitudes(l1)
            f1 = gi.FieldStream(spec.field_seed, 8, s.nchol)
            t1 = time.perf_counter()
            for _ in range(2):
                if free:
                    p1, l1, a1, _ = O.free_propagate(ham, p1, l1, a1, f1.next())
                else:
                    p1, w1, l1, _ = O.propagate(ham, p1, w1, l1, f1.next())
                O.local_energies(ham, p1)
            d1 = time.perf_counter() - t1
        single = {"value": 16 / d1, "cores": 1, "sample": f"8 walkers x 2 steps, {d1:.1f} s, BLAS limited to 1 thread"}
    except ImportError:
        pass
    return {"value": n_walkers * n_steps / dt, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
            "blas_threads": blas_threads, "cpu_model": cpu_model(), "single_thread": single,
            "sample": f"{n_walkers} walkers x {n_steps} {'free-projection ' if free else ''}steps "
                      f"(propagate + local energy, FP64) of {spec.name}, "
                      f"{dt:.1f} s on the host CPU, numpy complex128"}


def time_path(A, torch, ctx, spec, trial, xs, args):
    """Warm up, then time args.steps steps; returns timing, phases and walkers."""
    import afqmc_inputs as gi
    W = spec.nwalkers
    walkers = A.Walkers.from_numpy(gi.initial_walkers(trial, W))
    A.overlap(ctx, walkers)
    e_out = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
    free = args.projection == "free"
    est = torch.empty((1, A.FREE_EST if free else 4), dtype=torch.float64, device="cuda")
    amp = walkers.log_ovlp.clone()

    def step(k):
        reo = (k + 1) % spec.reortho_every == 0
        if free:
            if args.api == "step":
                A.free_step(ctx, walkers, xs[k], amp, e_out, est, reortho=reo)
                return
            A.free_propagate(ctx, walkers, xs[k], amp)
            if reo:
                A.reorthogonalize(ctx, walkers)
            A.local_energy(ctx, walkers, e_out)
            A.free_estimator(ctx, walkers, amp, e_out, est)
            return
        if args.api == "step":
            A.step(ctx, walkers, xs[k], e_out, est, reortho=reo)
            return
        A.propagate(ctx, walkers, xs[k])
        if reo:
            A.reorthogonalize(ctx, walkers)
        A.local_energy(ctx, walkers, e_out, est)

    nsteps = args.warmup + args.steps
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # the timed block, with the library's phase timers off
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.warmup, nsteps):
        step(k)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    h = est.cpu().numpy()[0]
    if free:
        energy = A.free_energy(h).real if h[9] > 0 else float("nan")
    else:
        energy = float(h[0] / h[1]) if h[1] > 0 else float("nan")
    flagged = int((walkers.flags.cpu().numpy() != 0).sum())
    # the phase breakdown from a block of its own (the per-phase events cost a
    # little time, so that block is not the one timed above)
    A.set_timing(ctx, True)
    for k in range(args.warmup, nsteps):
        step(k)
    torch.cuda.synchronize()
    phases = A.get_timings(ctx)
    A.set_timing(ctx, False)
    # further timed blocks (the same fields again), for the spread of the rate
    blocks = [total_ms]
    for _ in range(max(0, args.repeats)):
        torch.cuda.synchronize()
        ev0.record()
        for k in range(args.warmup, nsteps):
            step(k)
        ev1.record()
        torch.cuda.synchronize()
        blocks.append(ev0.elapsed_time(ev1))
    return {"total_ms": total_ms, "phases": phases, "walkers": walkers, "mixed_energy": energy,
            "flagged": flagged, "blocks_ms": blocks}


def bench_batching(args):
    print(json.dumps(batching_leg(args)), flush=True)
    return 0


def batching_leg(args, precisions=(("fp64", 0), ("fp32", 1))):
    """Aggregate throughput of the sixteen-system set, FP64 and FP32."""
    import numpy as np
    import torch
    import afqmc_inputs as gi
    from paper_2406_16238_amd import afqmc as A

    runs = gi.batching_specs()
    inputs = []
    for r in runs:
        h1, chol, ecore, trial = gi.make_system(r.system)
        inputs.append((A.SystemInput(h1, chol, ecore, trial, r.system.nalpha, r.system.nbeta, r.nwalkers, r.dt),
                       trial))
    total_w = sum(r.nwalkers for r in runs)
    nsteps = args.warmup + args.steps

    def buffers(idx):
        ws, xs, es = [], [], []
        for j in idx:
            sysin, trial = inputs[j]
            ws.append(A.Walkers.from_numpy(gi.initial_walkers(trial, sysin.nwalkers, seed=j)))
            xs.append(torch.empty((sysin.nwalkers, sysin.nchol), dtype=torch.float64, device="cuda"))
            es.append(torch.empty((sysin.nwalkers, 3), dtype=torch.complex128, device="cuda"))
        return ws, xs, es

    def timed(step_all, fill):
        for k in range(args.warmup):
            fill(k)
            step_all(k)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for k in range(args.warmup, nsteps):
            fill(k)
            step_all(k)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    gen = torch.Generator(device="cuda")

    def filler(xs):
        def fill(k):
            gen.manual_seed(1000 + k)
            for x in xs:
                x.normal_(generator=gen)
        return fill

    out_modes = {}
    for prec_name, prec in precisions:
        modes = {}
        # separate contexts, one after another on one stream
        ctxs = [A.setup_hamiltonian(inputs[j][0], A.default_options(precision=prec, streams=1))
                for j in range(len(inputs))]
        ws, xs, es = buffers(range(len(inputs)))
        for c, w in zip(ctxs, ws):
            A.overlap(c, w)

        def seq(k):
            for c, w, x, e in zip(ctxs, ws, xs, es):
                A.step(c, w, x, e, reortho=(k + 1) % 5 == 0)
        ms = timed(seq, filler(xs))
        modes["sequential"] = total_w * args.steps / (ms * 1e-3)
        for c in ctxs:
            c.close()
        del ctxs, ws, xs, es
        torch.cuda.empty_cache()
        for label, graph in (("streams", 0), ("streams+graph", 1)):
            ctx = A.setup_hamiltonian([i for i, _ in inputs], A.default_options(precision=prec, use_graph=graph))
            ws, xs, es = buffers(range(len(inputs)))
            A.overlap(ctx, ws)

            def together(k):
                A.step(ctx, ws, xs, es, reortho=(k + 1) % 5 == 0)
            ms = timed(together, filler(xs))
            modes[label] = total_w * args.steps / (ms * 1e-3)
            ctx.close()
            del ctx, ws, xs, es
            torch.cuda.empty_cache()
        out_modes[prec_name] = {k: round(v, 2) for k, v in modes.items()}
        out_modes[prec_name]["speedup_vs_sequential"] = round(max(modes["streams"], modes["streams+graph"]) /
                                                               modes["sequential"], 3)
    best = max(out_modes["fp64"]["streams"], out_modes["fp64"]["streams+graph"])
    out = {"metric": "aggregate walker-steps/s (propagate+energy), 16 uneven systems", "value": best,
           "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generator per system)",
           "config": {"workload": "batching-16-systems-M60-360", "nbasis": [r.system.nbasis for r in runs],
                      "nwalkers": [r.nwalkers for r in runs], "nchol": "4M", "n_per_spin": "M/10"},
           "modes": out_modes}
    return out


def train_cv_network(A, torch, ctx, trial, W, G, nsteps, epochs, seed0=5000):
    """Features and exact exchange along the path's own trajectory (fields drawn
    from seed0 on), then the network trained on them; returns the losses."""
    import afqmc_inputs as gi
    w = A.Walkers.from_numpy(gi.initial_walkers(trial, W))
    A.overlap(ctx, w)
    gen = torch.Generator(device="cuda")
    x = torch.empty((W, G), dtype=torch.float64, device="cuda")
    e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
    feats, eks = [], []
    for k in range(nsteps):
        gen.manual_seed(seed0 + k)
        x.normal_(generator=gen)
        A.step(ctx, w, x, e, reortho=(k + 1) % 5 == 0)
        f = torch.empty((W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
        q = torch.empty(W, dtype=torch.complex128, device="cuda")
        A.cv_collect(ctx, w, f, q)
        feats.append(f)
        eks.append(q)
    return A.cv_train(ctx, torch.cat(feats), torch.cat(eks), epochs, 256, 2e-3).cpu().numpy()


def stat_error_leg(A, torch, spec, nblocks=20, block_steps=10, equil_blocks=4, cv_train_steps=40, cv_epochs=30):
    """Mixed-estimator energies with stated statistical errors: the same
    walkers, fields and comb offsets run in blocks (comb and E_T feedback after
    each) through the FP64 path and each reduced or learned form; the per-step
    mixed energies after the first `equil_blocks` blocks are reblocked by the
    library (afqmc_reblock), and so is each form's per-step difference from
    FP64."""
    import numpy as np
    import afqmc_inputs as gi
    s = spec.system
    W, G = spec.nwalkers, s.nchol
    h1, chol, ecore, trial = gi.make_system(s)
    sysin = A.SystemInput(h1, chol, ecore, trial, s.nalpha, s.nbeta, W, spec.dt)
    del chol
    gen = torch.Generator(device="cuda")
    gen.manual_seed(spec.field_seed + 77)
    xb = torch.randn((nblocks, block_steps, W, G), dtype=torch.float64, device="cuda", generator=gen)
    offs = torch.rand((nblocks, 1), dtype=torch.float64, device="cuda", generator=gen)
    forms = {"fp64": dict(precision=A.FP64), "bf16x2": dict(precision=A.BF16X2_CONTRACT),
             "fp16t": dict(precision=A.FP16_TSPLIT_CONTRACT),
             "fp16t+fp32prop": dict(precision=A.FP16_TSPLIT_CONTRACT, prop_precision=A.FP32_CONTRACT),
             "cv_fp64": dict(precision=A.FP64, ex_mode=A.EX_CV)}
    series, rates, extra = {}, {}, {}
    for name, kw in forms.items():
        ctx = A.setup_hamiltonian(sysin, A.default_options(**kw))
        try:
            if kw.get("ex_mode") == A.EX_CV:
                losses = train_cv_network(A, torch, ctx, trial, W, G, cv_train_steps, cv_epochs)
                extra[name] = {"training_steps": cv_train_steps, "epochs": cv_epochs,
                               "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
            w = A.Walkers.from_numpy(gi.initial_walkers(trial, W))
            A.overlap(ctx, w)
            e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            est = torch.empty((nblocks, block_steps, 4), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for b in range(nblocks):
                A.run_block(ctx, w, xb[b], e, est[b], offs[b], step0=b * block_steps,
                            reortho_every=spec.reortho_every, feedback=True)
            ev1.record()
            torch.cuda.synchronize()
            rates[name] = W * nblocks * block_steps / (ev0.elapsed_time(ev1) * 1e-3)
            h = est.cpu().numpy().reshape(-1, 4)
            series[name] = h[:, 0] / h[:, 1]
        finally:
            ctx.close()
        torch.cuda.empty_cache()
    del xb
    skip = equil_blocks * block_steps

    def err(x):
        r = A.reblock(x[skip:])
        if r["optimal"] is not None:
            return r["mean"], r["std_err"], True
        # no level qualifies: the largest error of the levels with at least 8 blocks
        cand = [lv["std_err"] for lv in r["levels"] if lv["n"] >= 8]
        return r["mean"], max(cand) if cand else r["levels"][-1]["std_err"], False

    e64, s64, ok64 = err(series["fp64"])
    out = {"workload": spec.name, "nwalkers": W, "blocks": nblocks, "steps_per_block": block_steps,
           "equilibration_steps_excluded": skip, "population_control": "comb after each block",
           "e_shift_feedback": "block estimate", "error_analysis": "afqmc_reblock (Flyvbjerg-Petersen, "
           "Lee et al. level); difference errors from the reblocked per-step difference series",
           "fp64": {"energy_ha": e64, "err_ha": s64, "plateau": ok64, "walker_steps_per_s": round(rates["fp64"], 1)},
           "forms": {}}
    for name in forms:
        if name == "fp64":
            continue
        ef, sf, okf = err(series[name])
        dm, ds, okd = err(series[name] - series["fp64"])
        out["forms"][name] = {"energy_ha": ef, "err_form_ha": sf, "err_fp64_ha": s64, "diff_ha": dm,
                              "err_diff_ha": ds, "plateau": bool(okf and okd),
                              "within_0.1mHa": bool(abs(dm) <= 1e-4),
                              "walker_steps_per_s": round(rates[name], 1),
                              "speedup_vs_fp64": round(rates[name] / rates["fp64"], 3), **extra.get(name, {})}
    return out


def bench_cv(args):
    print(json.dumps(cv_leg(args, args.cv_system)), flush=True)
    return 0


def cv_leg(args, system):
    """Learned control variate: walker-steps/s with the exact exchange on a 1/8
    subset against full exchange, and the estimator's bias and spread at fixed
    walkers against plain subsampling (f = 0).  Headline shape, or the
    benzene-scale shape with its Cholesky tensor drawn on the device."""
    import numpy as np
    import torch
    import afqmc_inputs as gi
    from paper_2406_16238_amd import afqmc as A

    spec = gi.BENZENE_SCALE if system == "benzene" else gi.HEADLINE
    s = spec.system
    W, G = spec.nwalkers, s.nchol
    if s.recipe == "counter":
        h1, ecore, trial = gi.make_system_without_chol(s)
        chol = A.CholGen(G, s.seed, s.tau, s.scale_factor())
    else:
        h1, chol, ecore, trial = gi.make_system(s)
    sysin = A.SystemInput(h1, chol, ecore, trial, s.nalpha, s.nbeta, W, spec.dt)
    prec = PRECISION_CODE[args.precision]
    gen = torch.Generator(device="cuda")
    x = torch.empty((W, G), dtype=torch.float64, device="cuda")
    e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
    est = torch.empty((1, 4), dtype=torch.float64, device="cuda")

    def run(ctx, walkers, nsteps, seed0, hook=None):
        for k in range(nsteps):
            gen.manual_seed(seed0 + k)
            x.normal_(generator=gen)
            A.step(ctx, walkers, x, e, est, reortho=(k + 1) % 5 == 0)
            if hook:
                hook(k)

    def timed(ctx, walkers):
        run(ctx, walkers, args.warmup, 9000)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        run(ctx, walkers, args.steps, 9100)
        ev1.record()
        torch.cuda.synchronize()
        return W * args.steps / (ev0.elapsed_time(ev1) * 1e-3)

    out = {}
    t0 = time.time()
    ctx = A.setup_hamiltonian(sysin, A.default_options(precision=prec, ex_mode=A.EX_CV))
    setup_s = time.time() - t0
    # training samples: features and exact exchange along the path's own trajectory
    w = A.Walkers.from_numpy(gi.initial_walkers(trial, W))
    A.overlap(ctx, w)
    feats, eks = [], []

    def grab(k):
        f = torch.empty((W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
        q = torch.empty(W, dtype=torch.complex128, device="cuda")
        A.cv_collect(ctx, w, f, q)
        feats.append(f)
        eks.append(q)
    t0 = time.time()
    run(ctx, w, args.cv_train_steps, 5000, grab)
    losses = A.cv_train(ctx, torch.cat(feats), torch.cat(eks), args.cv_epochs, 256, 2e-3).cpu().numpy()
    out["training"] = {"steps": args.cv_train_steps, "samples": args.cv_train_steps * W, "epochs": args.cv_epochs,
                       "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                       "seconds": round(time.time() - t0, 2)}
    del feats, eks
    saved = [t.clone() for t in (w.phi, w.weight, w.log_ovlp, w.flags)]
    # estimator at fixed walkers: exact value from the full exchange, then R draws
    wt = w.weight.cpu().numpy()
    om = wt / wt.sum()
    fx = torch.empty((W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
    ex = torch.empty(W, dtype=torch.complex128, device="cuda")
    A.cv_collect(ctx, w, fx, ex)
    exact = float(np.sum(om * (fx[:, 0].cpu().numpy() + ex.cpu().numpy().real)))   # Re EJ + Re EK

    def draws(R):
        v = []
        for _ in range(R):
            A.local_energy(ctx, w, e)
            v.append(np.sum(om * e.cpu().numpy()[:, 2].real))
        return np.array(v)
    cvd = draws(args.cv_draws)
    params, norm = A.cv_get_params(ctx)
    zero = torch.zeros(A.CV_NPARAMS, dtype=torch.float32, device="cuda")
    # the method without the network: f = the training mean of EK (zero weights
    # keep only the target normalisation's mean), and plain subsampling (f = 0)
    A.cv_set_params(ctx, zero, norm)
    cmd = draws(args.cv_draws)
    A.cv_set_params(ctx, zero, torch.tensor([0.0] * A.CV_NFEAT + [1.0] * A.CV_NFEAT + [0.0, 0.0, 1.0, 1.0], dtype=torch.float64,
                                            device="cuda"))
    pld = draws(args.cv_draws)
    A.cv_set_params(ctx, params, norm)
    # throughput from the same walker state: control variate, then full exchange
    rates = {"control_variate": timed(ctx, A.Walkers(*[t.clone() for t in saved]))}
    ctx.close()
    torch.cuda.empty_cache()
    full = A.setup_hamiltonian(sysin, A.default_options(precision=prec))
    rates["full_exchange"] = timed(full, A.Walkers(*[t.clone() for t in saved]))
    full.close()
    k = -(-W // 8)
    out.update({
        "metric": f"walker-steps/s (propagate+energy) at M={s.nbasis},N={s.nalpha} with the learned exchange "
                  "control variate",
        "value": round(rates["control_variate"], 2), "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"{args.precision} (exchange, force bias) + f64 (rest)",
        "data": "synthetic (seeded generator" + ("; Cholesky tensor drawn on the device" if s.recipe == "counter"
                                                 else "") + "; network trained on the run's own trajectory)",
        "config": {"workload": spec.name, "nbasis": s.nbasis, "nalpha": s.nalpha, "nchol": G, "nwalkers": W,
                   "exact_exchange_walkers_per_call": k, "precision": args.precision,
                   "setup_seconds": round(setup_s, 1)},
        "full_exchange_value": round(rates["full_exchange"], 2),
        "speedup_vs_full_exchange": round(rates["control_variate"] / rates["full_exchange"], 3),
        "estimator_at_fixed_walkers": {
            "draws": args.cv_draws, "exact_e2_ha": exact,
            "cv_bias_ha": float(cvd.mean() - exact), "cv_stderr_ha": float(cvd.std(ddof=1) / np.sqrt(len(cvd))),
            "cv_spread_ha": float(cvd.std(ddof=1)),
            "constant_mean_bias_ha": float(cmd.mean() - exact), "constant_mean_spread_ha": float(cmd.std(ddof=1)),
            "plain_bias_ha": float(pld.mean() - exact), "plain_spread_ha": float(pld.std(ddof=1)),
            "variance_ratio_cv_over_constant_mean": float(cvd.var(ddof=1) / cmd.var(ddof=1)),
            "variance_ratio_cv_over_plain": float(cvd.var(ddof=1) / pld.var(ddof=1))}})
    return out


def medium_leg(args):
    """The FP64 path at the medium shape (M=200, N=20+20, G=800, 512 walkers):
    walker-steps/s and the FP64 exchange kernel's roofline."""
    import argparse as ap_
    import torch
    import afqmc_inputs as gi
    from paper_2406_16238_amd import afqmc as A
    spec = gi.MEDIUM
    s = spec.system
    W, G, M = spec.nwalkers, s.nchol, s.nbasis
    h1, chol, ecore, trial = gi.make_system(s)
    ctx = A.setup_hamiltonian(A.SystemInput(h1, chol, ecore, trial, s.nalpha, s.nbeta, W, spec.dt))
    del chol
    gen = torch.Generator(device="cuda")
    gen.manual_seed(spec.field_seed)
    xs = torch.randn((args.warmup + args.steps, W, G), dtype=torch.float64, device="cuda", generator=gen)
    a = ap_.Namespace(**vars(args))
    a.api, a.projection, a.repeats = "step", "phaseless", 0
    try:
        r = time_path(A, torch, ctx, spec, trial, xs, a)
    finally:
        ctx.close()
    return {"workload": spec.name, "dtype": "f64", "value": round(W * args.steps / (r["total_ms"] * 1e-3), 2),
            "unit": "walker-steps/s", "ms_per_step": round(r["total_ms"] / args.steps, 4),
            "mixed_energy": r["mixed_energy"], "roofline": exchange_roofline("fp64", r["phases"], M, s, G, W,
                                                                              spec.name)}


def run_legs(args):
    """The other workloads, compactly, for the same JSON line: the FP64 medium
    shape, reblocked energies of every form against FP64 (medium and headline),
    the sixteen-system set, and the learned control variate (headline and
    benzene scale)."""
    import argparse as ap_
    import torch
    import afqmc_inputs as gi
    from paper_2406_16238_amd import afqmc as A
    legs = {}
    a = ap_.Namespace(**vars(args))
    a.cv_train_steps, a.cv_epochs, a.cv_draws = args.cv_train_steps, args.cv_epochs, 40
    plan = [("medium_fp64", lambda: medium_leg(a)),
            ("stat_error_medium", lambda: stat_error_leg(A, torch, gi.MEDIUM)),
            ("stat_error_headline", lambda: stat_error_leg(A, torch, gi.HEADLINE)),
            ("batching", lambda: batching_leg(a, precisions=(("fp64", 0),))),
            ("cv_headline", lambda: cv_leg(a, "headline")),
            ("cv_benzene", lambda: cv_leg(a, "benzene"))]
    for name, fn in plan:
        t0 = time.time()
        print(f"leg {name} ...", file=sys.stderr, flush=True)
        try:
            legs[name] = fn()
        except Exception as ex:   # a failing leg is reported, not fatal to the line
            legs[name] = {"error": f"{type(ex).__name__}: {ex}"}
        legs[name]["leg_seconds"] = round(time.time() - t0, 1)
        print(f"leg {name} done in {legs[name]['leg_seconds']} s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return legs


def main(argv=None):
    args = parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the walker step on one GPU only; it offers no run on several GPUs "
              "(walkers would shard across GPUs with a 32-byte all-reduce per step).", file=sys.stderr)
        return 2

    if args.workload == "batching":
        return bench_batching(args)
    if args.workload == "cv":
        return bench_cv(args)
    if args.workload == "stat":
        import torch
        import afqmc_inputs as gi
        from paper_2406_16238_amd import afqmc as A
        for spec in (gi.MEDIUM, gi.HEADLINE):
            print(json.dumps(stat_error_leg(A, torch, spec)), flush=True)
        return 0

    import numpy as np
    import torch
    import afqmc_inputs as gi
    from paper_2406_16238_amd import afqmc as A

    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    spec = {"headline": gi.HEADLINE, "medium": gi.MEDIUM, "small": gi.SMALL}[args.workload]
    s = spec.system
    W, G, M = spec.nwalkers, s.nchol, s.nbasis
    h1, chol, ecore, trial = gi.make_system(s)
    sysin = A.SystemInput(h1, chol, ecore, trial, s.nalpha, s.nbeta, W, spec.dt)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(spec.field_seed)
    xs = torch.randn((args.warmup + args.steps, W, G), dtype=torch.float64, device="cuda", generator=gen)

    prop32 = args.prop_precision == "fp32"
    rep_key = args.precision + ("+fp32prop" if prop32 else "")
    forms = ["fp64"] if rep_key == "fp64" else ["fp64", rep_key]
    # the reported form with FP32 propagation too (the paper's mixed precision on top of it)
    p32_key = args.precision + "+fp32prop"
    p32_ok = s.nbasis % 4 == 0 and s.nalpha + s.nbeta <= 96
    if rep_key != "fp64" and not prop32 and not args.no_prop32_leg and p32_ok:
        forms.append(p32_key)
    # the split-BF16 form beside a trial-split one (the robust form at three products)
    alt_key = "bf16x2" if args.precision in ("fp16t", "bf16t") and not prop32 else None
    if alt_key:
        forms.append(alt_key)
    ctxs, runs = {}, {}
    for form in forms:
        prec_name = form.split("+")[0]
        opt = A.default_options(precision=PRECISION_CODE[prec_name])
        if form.endswith("+fp32prop"):
            opt.prop_precision = A.FP32_CONTRACT
        ctxs[form] = A.setup_hamiltonian(sysin, opt)
        runs[form] = time_path(A, torch, ctxs[form], spec, trial, xs, args)
    del chol

    rep = args.precision
    r = runs[rep_key]
    ms_per_step = r["total_ms"] / args.steps
    value = W * args.steps / (r["total_ms"] * 1e-3)
    # one exchange launch = one spin block of every walker (the phase timer
    # brackets each launch on the library's stream)
    roofline = exchange_roofline(rep, r["phases"], M, s, G, W, spec.name)
    free = args.projection == "free"
    step_tf = step_flops(M, s.nalpha, s.nbeta, G, free) * W / (ms_per_step * 1e-3) / 1e12

    out = {"metric": METRIC_FREE if free else METRIC, "value": round(value, 2), "unit": "walker-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": ("f64" if rep == "fp64" else
                     ("f16 (trial-split exchange, force bias)" if rep == "fp16t" else
                      f"{rep} (exchange, force bias)")) +
                    (" + f32 (V_HS, Taylor terms)" if prop32 else "") + ("" if rep_key == "fp64" else " + f64 (rest)"),
           "data": "synthetic (seeded generator: random symmetric h and Cholesky vectors scaled by "
                   "exp(-g/tau)/M, trial = lowest orbitals of a Fock-like matrix, N(0,1) fields)",
           "config": {"workload": spec.name, "nbasis": M, "nalpha": s.nalpha, "nbeta": s.nbeta, "nchol": G,
                      "nwalkers": W, "dt": spec.dt, "reortho_every": spec.reortho_every,
                      "precision": rep, "propagation": args.prop_precision, "taylor_order": 6, "api": args.api,
                      "projection": args.projection},
           "roofline": roofline,
           "step_algorithmic_tflops": round(step_tf, 3),
           "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in r["phases"].items()},
           "mixed_energy": round(r["mixed_energy"], 8), "walkers_flagged": r["flagged"],
           "repeat_blocks_walker_steps_per_s": [round(W * args.steps / (b * 1e-3), 1) for b in r["blocks_ms"]],
           "median_walker_steps_per_s": round(float(np.median([W * args.steps / (b * 1e-3) for b in r["blocks_ms"]])),
                                              2),
           "device": {"name": torch.cuda.get_device_name(0),
                      "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", "")}}
    if rep_key != "fp64":
        f = runs["fp64"]
        fp64_value = W * args.steps / (f["total_ms"] * 1e-3)
        # energy error of the reduced form on identical walker states: its own
        # final walkers evaluated by both paths
        e_lp = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        e_64 = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        A.local_energy(ctxs[rep_key], r["walkers"], e_lp)
        A.local_energy(ctxs["fp64"], r["walkers"], e_64)
        torch.cuda.synchronize()
        d = np.abs(e_lp.cpu().numpy()[:, 0] - e_64.cpu().numpy()[:, 0])
        out["speedup_vs_fp64"] = round(value / fp64_value, 3)
        out["fp64_path"] = {"value": round(fp64_value, 2), "ms_per_step": round(f["total_ms"] / args.steps, 4),
                            "exchange_ms_per_step": round(f["phases"]["exchange"][0] / args.steps, 4),
                            "mixed_energy": round(f["mixed_energy"], 8)}
        out["energy_error_vs_fp64_ha"] = {"max": float(d.max()), "rms": float(np.sqrt((d ** 2).mean())),
                                          "bar": 1e-4, "within_bar": bool(d.max() <= 1e-4)}
        # the same fields from the same walkers: the mixed estimators of the two trajectories
        out["mixed_energy_difference_vs_fp64_ha"] = abs(r["mixed_energy"] - f["mixed_energy"])
        out["fp64_path"]["roofline"] = exchange_roofline("fp64", f["phases"], M, s, G, W, spec.name)
    if p32_key in runs and p32_key != rep_key:
        q = runs[p32_key]
        e_q = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        e_64 = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        A.local_energy(ctxs[p32_key], q["walkers"], e_q)
        A.local_energy(ctxs["fp64"], q["walkers"], e_64)
        torch.cuda.synchronize()
        dq = np.abs(e_q.cpu().numpy()[:, 0] - e_64.cpu().numpy()[:, 0])
        qv = W * args.steps / (q["total_ms"] * 1e-3)
        out["fp32_propagation_path"] = {
            "value": round(qv, 2), "ms_per_step": round(q["total_ms"] / args.steps, 4),
            "speedup_vs_fp64": round(qv / (W * args.steps / (runs["fp64"]["total_ms"] * 1e-3)), 3),
            "energy_error_vs_fp64_ha": {"max": float(dq.max()), "bar": 1e-4, "within_bar": bool(dq.max() <= 1e-4)},
            "mixed_energy_difference_vs_fp64_ha": abs(q["mixed_energy"] - runs["fp64"]["mixed_energy"]),
            "note": "the reported form with V_HS and the Taylor terms in FP32 as well (the paper's mixed precision)"}
    if alt_key:
        q = runs[alt_key]
        e_q = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        e_64 = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        A.local_energy(ctxs[alt_key], q["walkers"], e_q)
        A.local_energy(ctxs["fp64"], q["walkers"], e_64)
        torch.cuda.synchronize()
        dq = np.abs(e_q.cpu().numpy()[:, 0] - e_64.cpu().numpy()[:, 0])
        qv = W * args.steps / (q["total_ms"] * 1e-3)
        out[f"{alt_key}_path"] = {
            "value": round(qv, 2), "ms_per_step": round(q["total_ms"] / args.steps, 4),
            "speedup_vs_fp64": round(qv / (W * args.steps / (runs["fp64"]["total_ms"] * 1e-3)), 3),
            "energy_error_vs_fp64_ha": {"max": float(dq.max()), "bar": 1e-4, "within_bar": bool(dq.max() <= 1e-4)},
            "mixed_energy_difference_vs_fp64_ha": abs(q["mixed_energy"] - runs["fp64"]["mixed_energy"]),
            "roofline": exchange_roofline(alt_key, q["phases"], M, s, G, W, spec.name),
            "note": "split BF16, two terms per operand and three products: accurate whatever the walkers' "
                    "distance from the trial"}
    if args.phases:
        for form in forms:
            print(f"-- {form}", file=sys.stderr)
            for k, (ms, n) in runs[form]["phases"].items():
                print(f"{k:12s} {ms / args.steps:9.3f} ms/step  {n:6d} launches", file=sys.stderr)
    for c in ctxs.values():
        c.close()
    del xs, runs
    torch.cuda.empty_cache()
    if not args.no_legs and args.workload == "headline" and args.projection == "phaseless":
        out["legs"] = run_legs(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_walkers, args.cpu_steps, free)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
