#!/usr/bin/env python
"""Throughput of the steric-constraint step on one MI355X.

One step = one whole pass of the hot path on the 100,000-rod suspension
(length 1, diameter 0.025, volume fraction 0.05, nematic: von Mises-Fisher
kappa = 20 about z; external forces and torques N(0,1); dt = 1e-4; pair
threshold 0.05 on the surface gap): directors, pair search, constraint
geometry, the BBPGD solve to residual 1e-8 and the Euler update.  Every step
starts from the same resident configuration (a device copy inside the timed
region), so each step does the same work.

Prints one JSON line: BBPGD iterations per second over the timed steps (the
whole step is timed, pair search included), LCP solves per second, the
roofline of the dominant solver kernel from HIP events sampled during the
timed steps, and the CPU oracle timed on a bounded sample.
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

METRIC = "BBPGD iters/sec and LCP solves/sec at 100k rods; HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bbpgd_rods100k.json")
TRAFFIC_FILE_400K = os.path.join(ROOT, "profiles", "traffic_bbpgd_rods400k.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2109_08206_amd", "csrc", f)
                  for f in ("rl_solver.hip", "rl_mixed.hip", "rl_device.hpp", "rl_internal.hpp")]


def kernel_bytes(n: int, nc: int) -> dict:
    """Algorithmic bytes per launch of the two BBPGD loop kernels: every array
    element the kernel must touch once (FP64 values, int32 indices).
    rod kernel:        per rod pptr+qptr 8, dir 24                    -> 32 n
                       per constraint, P side: (gamma, g) 16, (e, s_i) 32,
                       u_P write 8; Q side copy: (gamma, g) 16,
                       (e, s_j) 32, u_Q write 8                       -> 112 nc
    constraint kernel: per constraint qpos 4, u_P 8, u_Q 8, q 8,
                       (gamma, g) read 16 + write 16,
                       Q-side (gamma, g) write 16                     -> 76 nc"""
    return {"rod": 32 * n + 112 * nc, "con": 76 * nc}


def con_kernel_name(nc: int, fp32: bool = False) -> str:
    """The constraint kernel's instantiation for nc constraints: the library
    sizes its grid at about 2,048 constraints per workgroup (at least one, at
    most 512, or 256 in the mixed-precision solve, a multiple of 8) and takes
    256 threads with 8 constraints each
    (FP32) or 512 threads with 8 (FP64) once a workgroup's share exceeds
    2,048, else 512 threads with 4 (FP64) or 2 (FP32)."""
    g = min(max((nc + 2047) // 2048, 1), 256 if fp32 else 512)
    g = (g + 7) // 8 * 8
    wide = (nc + g - 1) // g > 2048
    if fp32:
        return "k_con32<256,8>" if wide else "k_con32<512,2>"
    return "k_con<2,512,8>" if wide else "k_con<2,512,4>"


def rod_lanes(n: int, nc: int) -> int:
    """Lanes per rod of the loop's rod kernel (three rounds of records each):
    eight above 8 constraints per rod (contact-only sets), else four."""
    return 8 if nc > 8 * n else 4


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, path: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on other kernel sources."""
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else float(k["hbm_bytes_per_launch"])


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_share() -> int:
    """Host threads this process may use: the CPUs it may run on, capped by
    OMP_NUM_THREADS when that is set (the share of the host a job gets)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(avail, int(omp))) if omp.isdigit() and int(omp) > 0 else avail


def cpu_baseline(sysm, iters: int) -> dict:
    """The sequential FP64 oracle timed on the host: its own source built
    -O3 -march=native for this CPU (the tests' checker build is -O2
    -ffp-contract=off).  One core on one system, then every core of the
    share at once, each thread solving the same problem independently
    (shared read-only inputs, its own work arrays; the oracle is sequential; ctypes releases the interpreter lock during
    the C call, so the threads run in parallel)."""
    import concurrent.futures as cf

    import oracle
    prev = oracle.use_build("timing")
    try:
        d = oracle.directors(sysm.quat)
        t0 = time.perf_counter()
        pr = oracle.pairs(sysm.x, d, 1.0, sysm.box, sysm.diam, sysm.cutoff)
        cs = oracle.assemble(sysm.x, d, 1.0, sysm.box, sysm.diam, sysm.eta, sysm.dt, pr, sysm.force)
        t1 = time.perf_counter()
        r = oracle.bbpgd(d, 1.0, sysm.diam, sysm.eta, pr, cs, tol=1e-8, max_iter=iters)
        t2 = time.perf_counter()
        # the start costs two products (g0 and the Cauchy step), like two iterations
        per_iter = (t2 - t1) / (r.iterations + 2)
        cores = _cpu_share()
        each = max(50, iters // 2)

        def one(_):
            ra = oracle.bbpgd(d, 1.0, sysm.diam, sysm.eta, pr, cs, tol=1e-8, max_iter=each)
            return ra.iterations + 2

        t3 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            done = sum(ex.map(one, range(cores)))
        t4 = time.perf_counter()
    finally:
        oracle.use_build(prev)
    return {"value": 1.0 / per_iter, "unit": "BBPGD iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{r.iterations} BBPGD iterations (+2 start products) of the sequential FP64 C oracle "
                      f"(-O3 -march=native) on the same {sysm.n}-rod system ({pr.n} constraints); pair search + "
                      f"assembly took {t1 - t0:.2f} s and are not in the rate",
            "all_cores": {"value": done / (t4 - t3), "unit": "BBPGD iters/s", "cores": cores,
                          "how": f"{cores} threads, each {each} iterations (+2) of its own solve of the problem, "
                                 f"{t4 - t3:.1f} s wall: aggregate throughput of independent solves"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "pairs_assembly_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 3)}


def _kernel_summary(prof, kb, names):
    avg = {"rod": prof["rod_ms"] / max(1, prof["rod_launches"]),
           "con": prof["con_ms"] / max(1, prof["con_launches"])}
    return avg, {names[k]: {"avg_us": 1e3 * avg[k], "alg_bytes": kb[k],
                            "alg_gbps": kb[k] / (avg[k] * 1e-3) / 1e9 if avg[k] > 0 else 0.0,
                            "samples": prof[f"{k}_launches"]} for k in ("rod", "con")}


def kernel_bytes32(n: int, nc: int) -> dict:
    """Algorithmic bytes per launch of the single-precision loop kernels.
    rod kernel:        per rod pptr+qptr 8, dir 24                    -> 32 n
                       per constraint, P and Q side: state 16 + (e, s) 16
                       + contact velocity write 4                     -> 72 nc
    constraint kernel: per constraint qpos 4, u_P 4, u_Q 4,
                       state read 16 + write 16, Q-side state
                       write 16                                       -> 60 nc"""
    return {"rod": 32 * n + 72 * nc, "con": 60 * nc}


def form_precision(args, torch, rl, rodsynth) -> dict:
    """FP64 against FP32-mixed whole steps on the precision workload."""
    dev = torch.device("cuda:0")
    n = args.rods if args.rods != 100_000 else 400_000
    phi = args.phi if args.phi else 0.08
    s = rodsynth.cfg_precision(args.seed, n=n, phi=phi)
    x0, q0 = torch.as_tensor(s.x, device=dev), torch.as_tensor(s.quat, device=dev)
    F, L = torch.as_tensor(s.force, device=dev), torch.as_tensor(s.length, device=dev)
    x, q = torch.empty_like(x0), torch.empty_like(q0)
    res = {}
    Us = {}
    for name, prec in (("fp64", rl.FP64), ("fp32_mixed", rl.FP32_MIXED)):
        slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        max_iter=200_000, precision=prec)
        U = torch.empty((s.n, 6), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            x.copy_(x0); q.copy_(q0)
            slv.step(x, q, L, F=F, U=U)
        slv.profile_enable(args.profile_every)
        slv.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, worst, status, npairs, refr = 0, 0.0, 0, 0, 0
        for _ in range(args.steps):
            x.copy_(x0); q.copy_(q0)
            _, info, npairs = slv.step(x, q, L, F=F, U=U)
            iters += info.iterations
            worst = max(worst, info.residual)
            status = max(status, info.status)
            refr += info.fp64_refreshes
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = slv.profile_read()
        slv.close()
        kb = (kernel_bytes if prec == rl.FP64 else kernel_bytes32)(s.n, npairs)
        ln = rod_lanes(s.n, npairs)
        names = {"rod": f"k_rod<2,false,3,{ln}>", "con": con_kernel_name(npairs)} if prec == rl.FP64 else \
            {"rod": f"k_rod32<false,3,{ln}>", "con": con_kernel_name(npairs, fp32=True)}
        avg, kern = _kernel_summary(prof, kb, names)
        dom = max(avg, key=avg.get)
        ach = kb[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
        res[name] = {"iters_per_s": iters / el, "ms_per_step": 1e3 * el / args.steps,
                     "iters_per_solve": iters / args.steps, "fp64_refreshes_per_solve": refr / args.steps,
                     "max_residual_fp64": worst, "status": status, "constraints": npairs,
                     "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": ach, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                  "traffic": (measured_traffic(dom + ("" if prec == rl.FP64 else "32"),
                                                               TRAFFIC_FILE_400K)
                                              if (s.n, args.seed, phi) == (400_000, 0, 0.08) else None),
                                  "alg_bytes_per_launch": kb[dom]},
                     "kernels": kern, "us_per_iteration": 1e3 * (avg["rod"] + avg["con"])}
        Us[name] = U.cpu()
    du = float(torch.linalg.norm(Us["fp32_mixed"] - Us["fp64"]) / torch.linalg.norm(Us["fp64"]))
    return {
        "metric": "precision form: FP32-mixed vs FP64 BBPGD, whole steps to residual 1e-8",
        "value": res["fp32_mixed"]["iters_per_s"], "unit": "BBPGD iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["fp32_mixed"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{s.n} rods L~U[0.5,1.5] d=0.025 isotropic phi={phi}, relaxed overlap-free "
                               f"start, one whole step to residual 1e-8",
                   "rods": s.n, "box": round(s.box, 4), "seed": args.seed},
        "fp64": res["fp64"], "fp32_mixed": res["fp32_mixed"],
        "speedup_per_iteration": res["fp64"]["us_per_iteration"] / max(1e-9, res["fp32_mixed"]["us_per_iteration"]),
        "speedup_per_step": res["fp64"]["ms_per_step"] / res["fp32_mixed"]["ms_per_step"],
        "U_rel_diff_fp32_mixed_vs_fp64": du,
    }


def form_batched(args, torch, rl, rodsynth) -> dict:
    """256 independent systems: one batched solve against one solve per system."""
    dev = torch.device("cuda:0")
    systems = rodsynth.cfg_batched(args.seed)
    pieces = {k: [] for k in ("dir", "pi", "pj", "e", "arm", "q", "F")}
    rods, pairs = [0], [0]
    singles = []
    for s in systems:
        slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8)
        x, quat, F = (torch.as_tensor(a, device=dev) for a in (s.x, s.quat, s.force))
        d = slv.directors(quat)
        pi, pj, img, _ = slv.build_pairs(x, d, 1.0)
        phi, e, arm, q = slv.assemble_D(x, d, 1.0, pi, pj, img, F)
        slv.close()
        singles.append((s, d, pi, pj, e, arm, q, F))
        for k, v in (("dir", d), ("pi", pi + rods[-1]), ("pj", pj + rods[-1]), ("e", e), ("arm", arm),
                     ("q", q), ("F", F)):
            pieces[k].append(v)
        rods.append(rods[-1] + s.n)
        pairs.append(pairs[-1] + pi.shape[0])
    cat = {k: torch.cat(v).contiguous() for k, v in pieces.items()}
    slv = rl.Solver(box=1.0, tol=1e-8, max_iter=200_000)
    slv.batch_tuning(0, 0)
    for _ in range(args.warmup):
        slv.solve_lcp_batched(rods, pairs, cat["dir"], 1.0, cat["pi"], cat["pj"], cat["e"], cat["arm"], cat["q"],
                              F=cat["F"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, U, infos = slv.solve_lcp_batched(rods, pairs, cat["dir"], 1.0, cat["pi"], cat["pj"], cat["e"],
                                            cat["arm"], cat["q"], F=cat["F"])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    used = slv.batch_tuning(0, 0)
    slv.close()
    iters = [i.iterations for i in infos]
    # the same systems one solve each
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_iters, Useq = 0, []
    for (s, d, pi, pj, e, arm, q, F) in singles:
        one = rl.Solver(box=s.box, tol=1e-8, max_iter=200_000)
        _, Ui, inf = one.solve_lcp(d, 1.0, pi, pj, e, arm, q, F=F)
        one.close()
        seq_iters += inf.iterations
        Useq.append(Ui)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    Useq = torch.cat(Useq)
    du = float(torch.linalg.norm(U - Useq) / torch.linalg.norm(Useq))
    S = len(systems)
    return {
        "metric": "batching form: independent systems solved to residual 1e-8 in one batched solve",
        "value": S / el, "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{S} periodic systems, rods log-uniform in [200, 20000], volume fraction "
                               f"uniform in [0.02, 0.1], isotropic, L=1, relaxed overlap-free starts",
                   "systems": S, "rods": rods[-1], "constraints": pairs[-1],
                   "seed": args.seed},
        "bbpgd_iters_per_s_aggregate": sum(iters) / el,
        "max_iterations_of_a_system": max(iters), "mean_iterations": sum(iters) / S,
        "statuses": {str(k): sum(1 for i in infos if i.status == k) for k in sorted({i.status for i in infos})},
        "max_residual": max(i.residual for i in infos),
        "workgroups_rod_con": list(used),
        "one_solve_per_system": {"seconds": el_seq, "systems_per_s": S / el_seq, "bbpgd_iters": seq_iters},
        "speedup_vs_one_per_system": el_seq / el,
        "U_rel_diff_vs_one_per_system": du,
    }


def form_adjoint(args, torch, rl, rodsynth) -> dict:
    """Gradient of sum |x_T|^2 (unwrapped centres) over a checkpointed rollout
    with respect to x0, theta0 and every step's forces, against the forward
    rollout alone."""
    import numpy as np

    from paper_2109_08206_amd.rollout import rollout
    dev = torch.device("cuda:0")
    n = args.rods if args.rods != 100_000 else 50_000
    s = rodsynth.cfg_rollout(args.seed, n=n)
    T, k = args.rollout_steps, args.checkpoint_every
    rng = np.random.default_rng([args.seed, 9])
    F = torch.empty((T, n, 6), dtype=torch.float64, device=dev)
    F[0] = torch.as_tensor(s.force, device=dev)
    for t in range(1, T):
        F[t] = torch.as_tensor(rng.standard_normal((n, 6)), device=dev)
    x0 = torch.as_tensor(s.x, device=dev)
    q0 = torch.as_tensor(s.quat, device=dev)
    slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000)

    def grad_run(steps):
        xg = x0.clone().requires_grad_(True)
        qg = q0.clone().requires_grad_(True)
        Fg = F[:steps].clone().requires_grad_(True)
        xu, _ = rollout(slv, xg, qg, 1.0, Fg, checkpoint_every=k, cg_tol=args.cg_tol, tape=not args.no_tape)
        loss = (xu * xu).sum()
        loss.backward()
        return xu, loss, xg, qg, Fg

    for _ in range(args.warmup):
        grad_run(min(T, 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        xu_f, _ = rollout(slv, x0, q0, 1.0, F, checkpoint_every=k, tape=not args.no_tape)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    xu, loss, xg, qg, Fg = grad_run(T)
    torch.cuda.synchronize()
    t_tot = time.perf_counter() - t0
    ctx = xu.grad_fn
    fwd_it = [i for i, _ in ctx.infos]
    adj = ctx.adjoint_infos
    slv.close()
    return {
        "metric": "differentiation form: gradient of sum |x_T|^2 over a checkpointed rollout (forward + backward)",
        "value": T / t_tot, "unit": "rollout steps/s with gradient", "n_gpus": 1, "steps": T,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_tot / T, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n} rods L=1 d=0.025 phi=0.05 isotropic, {T} steps, checkpoint every {k}, "
                               f"forward residual 1e-8, CG relative residual {args.cg_tol:g}",
                   "rods": n, "steps": T, "checkpoint_every": k, "seed": args.seed,
                   "gamma_tape": not args.no_tape},
        "forward_only_ms_per_step": 1e3 * t_fwd / T,
        "backward_ms_per_step": 1e3 * (t_tot - t_fwd) / T,
        "gradient_over_forward_time": t_tot / t_fwd,
        "mean_bbpgd_iterations": sum(fwd_it) / len(fwd_it),
        "mean_constraints": sum(p for _, p in ctx.infos) / len(ctx.infos),
        "mean_cg_iterations": sum(a.cg_iterations for a in adj) / len(adj),
        "max_cg_iterations": max(a.cg_iterations for a in adj),
        "mean_active": sum(a.n_active for a in adj) / len(adj),
        "cg_statuses": sorted({a.status for a in adj}),
        "loss": float(loss.detach()),
        "grad_norms": {"x0": float(xg.grad.norm()), "theta0": float(qg.grad.norm()), "F": float(Fg.grad.norm())},
        "forward_matches_gradient_run": bool(torch.equal(xu_f, xu.detach())),
    }


def form_kmc(args, torch, rl, rodsynth) -> dict:
    """Crosslinker kinetics on the paper-scale suspension: 400,000
    crosslinkers with the kinesin-5 parameters of the crosslinker table on
    the 100,000 nematic filaments, whole kinetics steps (filament binning and
    every crosslinker's transition) with the step's random numbers resident;
    then the coupled step of the method (kinetics, the doubly bound
    crosslinkers as links, the filament step with contacts, links and
    Brownian forces)."""
    dev = torch.device("cuda:0")
    s = rodsynth.cfg_paper_scale(args.seed)
    m = args.crosslinkers
    um3 = 602.214076
    kw = dict(eps=1625.0, Ka=90.9 / um3, koS=0.11, Ke=90.9 / um3, koD=0.11, kappa=300.0, rest=0.053, lam=0.258,
              kT=4.11e-3, rcs=0.039, rcd=0.11, dU=1.0)
    kp = rl.kmc_params(**kw)
    x = torch.as_tensor(s.x, device=dev)
    quat = torch.as_tensor(s.quat, device=dev)
    F = torch.as_tensor(s.force, device=dev)
    slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000)
    d = slv.directors(quat)
    state = torch.zeros(m, dtype=torch.int32, device=dev)
    rod = torch.full((m, 2), -1, dtype=torch.int32, device=dev)
    arc = torch.zeros((m, 2), dtype=torch.float64, device=dev)
    xl = torch.as_tensor(rodsynth.crosslinker_positions(m, s.box, args.seed), device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)

    def draws(k):
        return ([torch.rand((m, 4), dtype=torch.float64, device=dev, generator=gen) for _ in range(k)],
                [torch.randn((m, 3), dtype=torch.float64, device=dev, generator=gen) for _ in range(k)])

    # populate: steps of the same kinetics until the states settle
    us, xis = draws(args.kmc_populate)
    for k in range(args.kmc_populate):
        slv.kmc_step(x, d, 1.0, kp, state, rod, arc, xl, us[k], xis[k])
    us, xis = draws(args.warmup + args.steps)
    for k in range(args.warmup):
        slv.kmc_step(x, d, 1.0, kp, state, rod, arc, xl, us[k], xis[k])
    torch.cuda.synchronize()
    ev = [0] * 5
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        c = slv.kmc_step(x, d, 1.0, kp, state, rod, arc, xl, us[k], xis[k])
        ev = [a + b for a, b in zip(ev, c)]
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    occupancy = [int((state == k).sum()) for k in range(4)]
    # the coupled step: kinetics, links, filament step (contacts + links + Brownian)
    noise_gen = torch.Generator(device=dev)
    noise_gen.manual_seed(args.seed + 1)
    xs, qs = x.clone(), quat.clone()
    pipe = []
    nlinks = 0
    for k in range(3):
        u1, xi1 = draws(1)
        noise = torch.randn((s.n, 6), dtype=torch.float64, device=dev, generator=noise_gen)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dk = slv.directors(qs)
        slv.kmc_step(xs, dk, 1.0, kp, state, rod, arc, xl, u1[0], xi1[0])
        p, q, arm, kap, rest = slv.kmc_links(kp, state, rod, arc)
        nlinks = int(p.shape[0])
        _, info, _ = slv.step(xs, qs, 1.0, F=F, links=(p, q, arm, kap, rest, None), noise=noise, kT=kw["kT"])
        torch.cuda.synchronize()
        pipe.append(time.perf_counter() - t1)
    slv.close()
    out = {
        "metric": "crosslinker kinetics: crosslinker updates per second (binding/unbinding kinetic Monte Carlo)",
        "value": m / el, "unit": "crosslinker updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{m} crosslinkers (kinesin-5 parameters of the crosslinker table: eps 1625/um, "
                               f"K_a = K_e = 90.9/uM, k_o = 0.11/s, kappa 300 pN/um, l_o 53 nm, lambda 0.258, "
                               f"r_cs 39 nm, r_cd 110 nm) on {s.n} filaments L=1 phi=0.05 nematic vMF kappa=20",
                   "crosslinkers": m, "rods": s.n, "box": round(s.box, 4), "seed": args.seed},
        "states_U_SA_SB_D": occupancy, "events_per_step": [e / args.steps for e in ev],
        "coupled_step": {"ms": [round(1e3 * v, 3) for v in pipe], "links": nlinks,
                         "what": "kinetics + links of the doubly bound + filament step (contacts, links, "
                                 "Brownian force) to residual 1e-8",
                         "last_status": info.status, "last_iterations": info.iterations},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = kmc_cpu_baseline(s, kw, state, rod, arc, xl)
    return out


def form_dynamics(args, torch, rl, rodsynth) -> dict:
    """Whole coupled steps of a confined, crosslinked suspension: 100,000
    rods of length 1 in a spherical shell at the density of the paper's
    confined suspension (3,200 rods in a shell of radius 3 um, so radius
    3 (n/3200)^(1/3)), 400,000 kinesin-5 crosslinkers inside the shell,
    each step being the crosslinker
    kinetics, the doubly bound crosslinkers as links, and the filament step
    with contacts, links and the shell as one constraint set, Brownian
    forces, a warm start from the previous step and the virial stress.  The
    random numbers of every step are drawn before the timed region."""
    dev = torch.device("cuda:0")
    n, m = args.rods, args.crosslinkers
    radius = 3.0 * (n / 3200.0) ** (1.0 / 3.0)
    s = rodsynth.confined_system(n, seed=args.seed, radius=radius)
    wl = [rodsynth.shell_wall(s, radius)]
    um3 = 602.214076
    kT = 4.11e-3
    kw = dict(eps=1625.0, Ka=90.9 / um3, koS=0.11, Ke=90.9 / um3, koD=0.11, kappa=300.0, rest=0.053, lam=0.258,
              kT=kT, rcs=0.039, rcd=0.11, dU=1.0)
    kp = rl.kmc_params(**kw)
    x = torch.as_tensor(s.x, device=dev)
    quat = torch.as_tensor(s.quat, device=dev)
    F = torch.as_tensor(s.force, device=dev)
    slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000)
    state = torch.zeros(m, dtype=torch.int32, device=dev)
    rod = torch.full((m, 2), -1, dtype=torch.int32, device=dev)
    arc = torch.zeros((m, 2), dtype=torch.float64, device=dev)
    c = 0.5 * s.box
    xl = torch.as_tensor(rodsynth.crosslinker_positions_ball(m, (c, c, c), radius, args.seed), device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    total = args.kmc_populate + args.warmup + args.steps
    us = [torch.rand((m, 4), dtype=torch.float64, device=dev, generator=gen) for _ in range(total)]
    xis = [torch.randn((m, 3), dtype=torch.float64, device=dev, generator=gen) for _ in range(total)]
    noise = [torch.randn((n, 6), dtype=torch.float64, device=dev, generator=gen) for _ in range(args.warmup + args.steps)]
    d = slv.directors(quat)
    for k in range(args.kmc_populate):
        slv.kmc_step(x, d, 1.0, kp, state, rod, arc, xl, us[k], xis[k])

    def coupled(k):
        dk = slv.directors(quat)
        slv.kmc_step(x, dk, 1.0, kp, state, rod, arc, xl, us[args.kmc_populate + k], xis[args.kmc_populate + k])
        p, q, arm, kap, rest, key = slv.kmc_links(kp, state, rod, arc, keys=True)
        _, info, npairs = slv.step(x, quat, 1.0, F=F, links=(p, q, arm, kap, rest, None, key), walls=wl,
                                   noise=noise[k], kT=kT, warm_start=not args.cold_start, stress=True)
        return info, npairs, int(p.shape[0]), slv.last_wall_contacts

    for k in range(args.warmup):
        coupled(k)
    slv.profile_enable(args.profile_every)
    slv.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, status, res = [], 0, 0.0
    counts = []
    for k in range(args.warmup, args.warmup + args.steps):
        info, npairs, nlinks, nwall = coupled(k)
        iters.append(info.iterations)
        status = max(status, info.status)
        res = max(res, info.residual)
        counts.append((npairs, nlinks, nwall))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = slv.profile_read()
    slv.profile_enable(0)
    stress = slv.last_stress
    slv.close()
    npairs, nlinks, nwall = counts[-1]
    nc = npairs + nlinks + nwall
    nq = npairs + nlinks
    # general-mode loop kernels: the contact-only records plus per rod its two
    # split indices (8 B) and per constraint the compliance (8 B); a wall
    # constraint has no Q side
    kb = {"rod": 40 * n + 56 * nc + 56 * nq, "con": 60 * nc + 24 * nq}
    avg = {"rod": prof["rod_ms"] / max(1, prof["rod_launches"]),
           "con": prof["con_ms"] / max(1, prof["con_launches"])}
    names = {"rod": "k_rod<2,true,gen,3,4>", "con": con_kernel_name(nc)[:-1] + ",gen>"}
    dom = max(avg, key=avg.get)
    achieved = kb[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    return {
        "metric": "dynamics form: coupled steps per second (crosslinker kinetics, then contacts, crosslinker links "
                  "and the confining shell as one constraint set with Brownian forces, warm-started, with the "
                  "virial stress)",
        "value": args.steps / el, "unit": "coupled steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n} rods L=1 d=0.025 in a spherical shell of radius {radius:.3f} (the density of "
                               f"the paper's 3,200 rods in radius 3), "
                               f"isotropic; {m} kinesin-5 crosslinkers in the shell; kT 4.11e-3 pN um; dt 1e-4 s",
                   "rods": n, "crosslinkers": m, "radius": round(radius, 4), "seed": args.seed,
                   "warm_start": not args.cold_start},
        "bbpgd_iters_per_s": sum(iters) / el, "iterations_per_step": iters, "max_residual": res, "status": status,
        "constraints_last_step": {"contacts": npairs, "links": nlinks, "wall": nwall},
        "stress_trace_last_step": {"contacts": float(stress[0].trace()), "links": float(stress[1].trace())},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": kb[dom], "avg_launch_us": 1e3 * avg[dom]},
        "kernels": {names[k]: {"avg_us": 1e3 * avg[k], "alg_bytes": kb[k],
                               "alg_gbps": kb[k] / (avg[k] * 1e-3) / 1e9 if avg[k] > 0 else 0.0,
                               "samples": prof[f"{k}_launches"]} for k in ("rod", "con")},
    }


def kmc_cpu_baseline(s, kw, state, rod, arc, xl) -> dict:
    """The oracle's kinetics step (every crosslinker against every
    filament) on 2,000 crosslinkers sampled across the four states."""
    import numpy as np

    import oracle
    prev = oracle.use_build("timing")
    try:
        st = state.cpu().numpy()
        rng = np.random.default_rng(0)
        pick = np.concatenate([rng.choice(np.flatnonzero(st == k), min(500, int((st == k).sum())), replace=False)
                               for k in range(4) if (st == k).any()])
        sub = oracle.Crosslinkers(st[pick].copy(), rod.cpu().numpy()[pick].copy(),
                                  np.ascontiguousarray(arc.cpu().numpy()[pick]),
                                  np.ascontiguousarray(xl.cpu().numpy()[pick]))
        ko = oracle.kmc_params(diam=s.diam, dt=s.dt, **kw)
        vbd = oracle.kmc_effective_volume(ko)
        d = oracle.directors(s.quat)
        u = rng.random((pick.size, 4))
        xi = rng.standard_normal((pick.size, 3))
        t0 = time.perf_counter()
        oracle.kmc_step(s.x, d, 1.0, s.box, ko, vbd, sub, u, xi)
        el = time.perf_counter() - t0
    finally:
        oracle.use_build(prev)
    return {"value": pick.size / el, "unit": "crosslinker updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one kinetics step of {pick.size} crosslinkers (500 per state) against all {s.n} filaments "
                      f"(the oracle tests every filament), {el:.2f} s, -O3 -march=native",
            "cpu_model": _cpu_model()}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rods", type=int, default=100_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--profile-every", type=int, default=32, help="sample kernel events every k-th iteration (each sample costs a few us of launch overhead)")
    ap.add_argument("--cpu-iters", type=int, default=800, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", choices=["step", "precision", "batched", "adjoint", "kmc", "dynamics"], default="step",
                    help="step: the FP64 whole-step benchmark (default); precision: FP32-mixed vs FP64; "
                         "batched: many systems in one batched solve; adjoint: gradient of a rollout; "
                         "kmc: crosslinker kinetics; dynamics: coupled steps of a confined, crosslinked, "
                         "Brownian suspension")
    ap.add_argument("--rollout-steps", type=int, default=100, help="adjoint form: rollout length")
    ap.add_argument("--checkpoint-every", type=int, default=10, help="adjoint form: checkpoint interval")
    ap.add_argument("--cg-tol", type=float, default=1e-10, help="adjoint form: CG relative residual")
    ap.add_argument("--no-tape", action="store_true",
                    help="adjoint form: re-solve each step cold in the backward pass instead of replaying gamma")
    ap.add_argument("--phi", type=float, default=None, help="volume fraction override (precision form)")
    ap.add_argument("--crosslinkers", type=int, default=400_000, help="kmc form: crosslinkers")
    ap.add_argument("--kmc-populate", type=int, default=50, help="kmc form: untimed steps that populate the states")
    ap.add_argument("--cold-start", action="store_true", help="dynamics form: every solve from zero forces")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy a 1 GiB device buffer once (reference for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        return 2

    import torch

    import paper_2109_08206_amd as rl
    import rodsynth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.form == "precision":
        print(json.dumps(form_precision(args, torch, rl, rodsynth)), flush=True)
        return 0
    if args.form == "batched":
        print(json.dumps(form_batched(args, torch, rl, rodsynth)), flush=True)
        return 0
    if args.form == "adjoint":
        print(json.dumps(form_adjoint(args, torch, rl, rodsynth)), flush=True)
        return 0
    if args.form == "kmc":
        print(json.dumps(form_kmc(args, torch, rl, rodsynth)), flush=True)
        return 0
    if args.form == "dynamics":
        print(json.dumps(form_dynamics(args, torch, rl, rodsynth)), flush=True)
        return 0
    dev = torch.device("cuda:0")
    s = rodsynth.cfg_paper_scale(args.seed, n=args.rods)
    x0 = torch.as_tensor(s.x, device=dev)
    q0 = torch.as_tensor(s.quat, device=dev)
    F = torch.as_tensor(s.force, device=dev)
    x, q = torch.empty_like(x0), torch.empty_like(q0)
    U = torch.empty((s.n, 6), dtype=torch.float64, device=dev)
    slv = rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000)

    def one_step():
        x.copy_(x0)
        q.copy_(q0)
        return slv.step(x, q, 1.0, F=F, U=U)

    for _ in range(args.warmup):
        one_step()
    slv.profile_enable(args.profile_every)
    slv.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, npairs, res, status = 0, 0, 0.0, 0
    for _ in range(args.steps):
        _, info, npairs = one_step()
        iters += info.iterations
        res = max(res, info.residual)
        status = max(status, info.status)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = slv.profile_read()
    slv.profile_enable(0)

    elapsed = t1 - t0
    kb = kernel_bytes(s.n, npairs)
    avg = {"rod": prof["rod_ms"] / max(1, prof["rod_launches"]),
           "con": prof["con_ms"] / max(1, prof["con_launches"])}
    names = {"rod": f"k_rod<2,true,3,{rod_lanes(s.n, npairs)}>", "con": con_kernel_name(npairs)}
    dom = max(avg, key=avg.get)
    achieved = kb[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    traffic = measured_traffic(dom)
    per_iter_bytes = kb["rod"] + kb["con"]
    out = {
        "metric": METRIC,
        "value": iters / elapsed,
        "unit": "BBPGD iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.n} rods L=1 d=0.025 phi=0.05 nematic vMF kappa=20, one whole step to "
                               f"residual 1e-8 (pairs + geometry + BBPGD + update)",
                   "rods": s.n, "constraints": npairs, "box": round(s.box, 4), "seed": args.seed},
        "lcp_solves_per_s": args.steps / elapsed,
        "iters_per_solve": iters / args.steps,
        "max_residual": res,
        "status": status,
        "solver_alg_gbps": per_iter_bytes * iters / elapsed / 1e9,
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": kb[dom], "avg_launch_us": 1e3 * avg[dom]},
        "kernels": {names[k]: {"avg_us": 1e3 * avg[k], "alg_bytes": kb[k],
                               "alg_gbps": kb[k] / (avg[k] * 1e-3) / 1e9 if avg[k] > 0 else 0.0,
                               "samples": prof[f"{k}_launches"]} for k in ("rod", "con")},
    }
    slv.close()
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_iters)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
