#!/usr/bin/env python3
"""Benchmark: stochastic disconnected loops on a 16^3 x 32 lattice (one GPU).

Workload (the paper's lattice shape, Sec. II; synthetic links stand in for
its SESAM ensemble): U = exp(i eps H) with eps = 0.6, kappa = 0.1596 (about
400 FP64 BiCGStab iterations to 1e-12), antiperiodic time; Z4 noise with
spin-colour-time dilution, 12 x 32 = 384 diluted sources per noise vector.
One step = one noise vector: noise generation, even-odd preparation, 384
batched Schur solves to |Dx-b|/|b| <= 1e-12 (CGNR iteration in FP32
arithmetic on 16-bit fixed-point vectors and links, FP64 reliable updates;
--prec f32 stores FP32), odd-site reconstruction and the contraction of
Eq. (loop stochastic) for Gamma = 1, g5, g1..g4.

Prints one JSON line:  value = diluted solves per second (whole job).
roofline: the dominant kernel of the step, the one of the iteration's
timed kernels with the largest summed time (events around every launch on
the library's stream): the first hop H_oe (algorithmic bytes = 8 links per
site + input + output per site and right-hand side), the hop with the fused
epilogue that ends each CGNR iteration (+ its two own-site operands), or
the vector update of x and p (5 fields); roofline_by_kernel: all three.  cpu_baseline: the FP64 oracle solving one of the
same diluted sources on the host cores.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Wilson solves/sec + dslash HBM GB/s at 16^3x32; loop rel. err vs FP64"
HBM_PEAK_GBS = 8000.0
# published FP32 vector peak: 256 CUs x 4 SIMDs x 32 FMA lanes per cycle x
# 2 flop x 2.4 GHz; plain (non-packed) FP32 FMA, add and multiply issue at
# that rate (one wave64 instruction per 2 cycles), conversions and 16-bit
# integer work at half of it
FP32_PEAK_TFLOPS = 157.3
FLOP_PER_SITE = 1320  # standard count of one hopping term per output site and right-hand side
SITE_BYTES = {"f32": 96, "bf16": 96, "h16": 52}
LINK_BYTES = {"f32": 48, "bf16": 24, "h16": 24}
# rocprofv3 counter summary of the hopping kernels timed here (FETCH_SIZE and
# WRITE_SIZE passes, scaled by a copy kernel of known size); their traffic is
# reported only while the kernel sources still hash to the recorded value
def traffic_profile(prec):
    return os.path.join(ROOT, "profiles", f"hopping_{prec}r12_stoch_16x16x16x32.md")


# the timed kernels of the iteration: library profiling slot, the vector
# fields each reads or writes once per site and right-hand side (CGNR), and
# whether it reads the links (a hop)
HOPS = {"first_hop": (0, 2, True), "end_hop": (1, 4, True), "vector_update": (2, 5, False)}


def kernel_source_hash():
    """SHA-256 over the HIP sources and the C header, in sorted path order."""
    from paper_1108_2473_amd import build
    return build.source_hash()


def profiled_traffic(prec, hop="first_hop"):
    """HBM bytes per launch of one timed hop from the committed counter
    summary, or None if the summary is missing or was taken on other kernel
    sources."""
    try:
        txt = open(traffic_profile(prec)).read()
    except OSError:
        return None
    key = "traffic_bytes_per_launch" + ("" if hop == "first_hop" else "_" + hop)
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    m_t = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_t or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_t.group(1))


def window(tag, t0_ns):
    """Log a monotonic-clock interval (the clock of rocprofv3's kernel
    timestamps) ending now, so that a kernel trace of the run can be cut to
    the workload it brackets."""
    log(f"[bench] window {tag} {t0_ns} {time.monotonic_ns()}")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# vector passes (fields read or written once per site and right-hand side) of
# one Krylov iteration, besides the links: CGNR with the carried normal
# residual: q = Dhat p (hop 2 + hop with p own and q out 3), z -= alpha Dhat^+ q
# (hop 2 + hop with q own, z own and z out 4), x += alpha p, p = z + beta p
# (p, z, x in; x, p out: 5); BiCGStab: Dhat p with <r0, v> (2 + 4), s = r -
# alpha v (3), Dhat s with <t, s>, |t|^2 (2 + 3), x and r update (5 in, 2 out),
# p update (3 in, 1 out)
ITER_PASSES = {"cgnr": 16, "bicgstab": 25}
ITER_HOPS = 4  # hopping launches per iteration, each reading the links of every site once


def iteration_roofline(solver, prec, Vh, system_iterations, launches_per_step, seconds_per_step):
    """Algorithmic bytes of the Krylov iteration kernels of one step (vector
    passes per system-iteration and site, links once per hopping launch) over
    the whole step's time: the rate of the iteration as a whole, replacements,
    host checks, noise and contraction included in the time only."""
    vec = ITER_PASSES[solver] * SITE_BYTES[prec] * Vh * system_iterations
    lnk = 8 * LINK_BYTES[prec] * Vh * launches_per_step
    gbs = (vec + lnk) / seconds_per_step / 1e9
    return {"bytes_per_site_and_system_iteration": ITER_PASSES[solver] * SITE_BYTES[prec],
            "system_iterations_per_step": system_iterations, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def cpu_model():
    """Model name of the host CPU (/proc/cpuinfo), or the platform string."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(U, b, x_mp, dims, bc, kappa, gam):
    """The FP64 oracle (even-odd BiCGStab, OpenMP over sites) on a bounded
    sample of the workload: two of its diluted sources solved to 1e-12 with
    every thread of the process, then the same solver single-threaded for 40
    iterations of one source, its per-iteration time scaled to the threaded
    run's iteration count.  Returns (cpu_baseline dict, loop error of the
    mixed-precision GPU solution of b[0] against the oracle's)."""
    import numpy as np
    import oracle as O
    ncpu = 2
    nthr = O.num_threads()
    t2 = time.perf_counter()
    x_or, it_or, res_or, fails = O.solve(U, b[:ncpu], dims, bc, kappa, tol=1e-12, max_iter=1200)
    t_or = time.perf_counter() - t2
    if fails:
        raise SystemExit(f"oracle baseline: {fails} solves missed 1e-12")
    n1 = 40
    O.set_num_threads(1)
    try:
        t3 = time.perf_counter()
        O.solve(U, b[:1], dims, bc, kappa, tol=1e-12, max_iter=n1)
        t_1 = time.perf_counter() - t3
    finally:
        O.set_num_threads(nthr)
    it_mean = float(np.mean(it_or[:ncpu]))
    rate_1 = 1.0 / (t_1 / n1 * it_mean)
    cpu = {"value": ncpu / t_or, "unit": "solves/s", "cores": nthr, "kind": "oracle",
           "cpu_model": cpu_model(),
           "single_thread_value": rate_1,
           "sample": f"{ncpu} spin-colour-time diluted Z4 sources of the same 16^3x32 workload (timeslices 0 "
                     f"and 5) solved by the FP64 oracle (even-odd BiCGStab, "
                     f"{'/'.join(str(int(v)) for v in it_or[:ncpu])} iterations, |Dx-b|/|b| <= "
                     f"{max(res_or[:ncpu]):.1e}) in {t_or:.1f} s on {nthr} threads; single-threaded: "
                     f"{n1} iterations of one source in {t_1:.1f} s, scaled to {it_mean:.0f} iterations "
                     f"per solve"}
    # loop error vs FP64: this source's contribution eta^+ Gamma phi on its timeslice
    Vs = dims[0] * dims[1] * dims[2]
    e = b[0, :Vs]
    errs = []
    l1 = None
    for g in gam:
        G = O.gamma(g)
        lg = np.einsum("sac,ab,sbc->s", e.conj(), G, x_mp[0, :Vs])
        lo = np.einsum("sac,ab,sbc->s", e.conj(), G, x_or[0, :Vs])
        if l1 is None:
            l1 = np.abs(lo).max()
        errs.append(np.abs(lg - lo).max() / l1)
    loop_err = max(errs)
    log(f"[bench] oracle {t_or:.1f}s for {ncpu} solves ({nthr} threads), single thread {rate_1:.4f} solves/s "
        f"(extrapolated); loop rel err vs FP64 {loop_err:.2e}")
    return cpu, loop_err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["f32", "bf16", "h16"], default="h16")
    ap.add_argument("--batch", type=int, default=384)
    ap.add_argument("--solver", choices=["cgnr", "bicgstab"], default="cgnr")
    ap.add_argument("--delta", type=float, default=0.0, help="reliable-update trigger (0: the library default)")
    ap.add_argument("--lds", type=int, default=-1,
                    help="LDS mode of the hopping kernel (-1: the library default; 3: packed 16-bit hop)")
    ap.add_argument("--rt", type=int, default=0, help="right-hand sides per workgroup (0: the library default)")
    ap.add_argument("--group", type=int, default=0,
                    help="right-hand-side blocks that sweep the site blocks together (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the other workloads (exact loops, uneven TSM batch, gradient)")
    ap.add_argument("--fp64-rhs", type=int, default=4, help="single-RHS FP64 GPU solves for the reference rate")
    ap.add_argument("--timed-only", action="store_true",
                    help="run only the warmup and timed steps (for kernel profiles of the timed region)")
    ap.add_argument("--metrics-jsonl", default="",
                    help="append one JSON line per timed solve (iterations, replacements, residual) to this file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device before the timed steps (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards over "
              "independent sources and needs no multi-GPU run here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1108_2473_amd as fl
    import synth_inputs as S

    W = S.WORKLOADS["stoch_16x16x16x32"]
    dims, eps, kappa, bc = W["dims"], W["eps"], W["kappa"], W["bc_t"]
    gam = fl.GAMMAS_PAPER
    log(f"[bench] links {dims} eps={eps} kappa={kappa}")
    U = S.random_links(dims, eps, W["link_seed"])
    lat = fl.Lattice(dims, bc, device=0)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    prec = {"f32": fl.PREC_F32, "bf16": fl.PREC_BF16, "h16": fl.PREC_H16}[args.prec]
    solver = fl.SOLVER_CGNR if args.solver == "cgnr" else fl.SOLVER_BICGSTAB
    lp = fl.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, batch=args.batch, solver=solver,
                         delta=args.delta)
    if args.lds != -1 or args.rt or args.group:
        lat.set_tile(prec=prec, gauge_reals=12, rt=args.rt, group=args.group, lds=args.lds)
    nt = dims[3]
    solves_per_step = 12 * nt

    def step(r):
        q = fl.NoiseParams(noise=fl.NOISE_Z4, seed=W["noise_seed"], r0=r, n_lp=1, n_hp=0,
                           dilution=fl.DIL_TIME | fl.DIL_SPIN | fl.DIL_COLOUR, t_begin=0, t_end=nt)
        return lat.loops_stochastic(q, gam, lp=lp)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for k in range(args.warmup):
        t0 = time.perf_counter()
        step(1000 + k)
        log(f"[bench] warmup step {k}: {time.perf_counter() - t0:.2f}s")
    for slot, _, _ in HOPS.values():
        lat.profile_enable(slot, True)
    torch.cuda.synchronize()
    w_steps = time.monotonic_ns()
    t0 = time.perf_counter()
    loops = []
    solve_stats = []
    for k in range(args.steps):
        loops.append(step(k))
        solve_stats.append(lat.last_stats())  # host copy of the call's statistics (no device work)
        log(f"[bench] step {k} done at {time.perf_counter() - t0:.2f}s "
            f"({lat.profile_read(fl.PROF_DSLASH)['launches']} hopping launches so far)")
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    window("timed_steps", w_steps)
    # every timed solve must have met the stopping rule on the full operator
    conv = np.concatenate([st["converged"] for st in solve_stats])
    resid = np.concatenate([st["true_resid"] for st in solve_stats])
    iters = np.concatenate([st["iters"] for st in solve_stats])
    upd = np.concatenate([st["updates"] for st in solve_stats])
    if len(conv) != solves_per_step * args.steps or not conv.all() or not (resid <= 1e-12).all():
        raise SystemExit(f"bench: {int((~conv).sum())} of {len(conv)} timed solves missed 1e-12 "
                         f"(largest residual {resid.max():.3e})")
    solves_summary = {"solves": int(len(conv)), "converged": int(conv.sum()),
                      "max_true_resid_full_operator": float(resid.max()),
                      "iterations_mean": round(float(iters.mean()), 1), "iterations_max": int(iters.max()),
                      "fp64_updates_mean": round(float(upd.mean()), 2)}
    log(f"[bench] timed solves: {solves_summary}")
    if args.metrics_jsonl:
        for k, st in enumerate(solve_stats):
            fl.append_jsonl(args.metrics_jsonl, fl.stats_records(st, step=k, workload="stochastic_16x16x16x32",
                                                                 prec=args.prec, solver=args.solver))
    profs = {}
    for name, (slot, _, _) in HOPS.items():
        pr = lat.profile_read(slot)
        lat.profile_enable(slot, False)
        pr["avg_us"] = pr["ms"] * 1e3 / max(1, pr["launches"])
        pr["achieved"] = pr["bytes"] / (pr["ms"] * 1e-3) / 1e9 if pr["ms"] > 0 else 0.0
        profs[name] = pr
    # the roofline is reported for the kernel of the iteration that takes
    # the most time (the two epilogue-free hops and the end hop, the vector
    # update; nothing else comes near them)
    dominant = max(profs, key=lambda h: profs[h]["ms"])
    prof = profs["first_hop"]
    achieved, avg_us = prof["achieved"], prof["avg_us"]
    value = solves_per_step * args.steps / T
    log(f"[bench] {value:.1f} solves/s; hopping kernel {prof['launches']} launches, avg {avg_us:.1f} us, "
        f"{achieved:.0f} GB/s; end hop avg {profs['end_hop']['avg_us']:.1f} us, "
        f"{profs['end_hop']['achieved']:.0f} GB/s; vector update avg {profs['vector_update']['avg_us']:.1f} us, "
        f"{profs['vector_update']['achieved']:.0f} GB/s; dominant: {dominant}")

    # disconnected two-point function (Eq. all_dis_corr) from the timed steps
    # loops: two independent noise vectors, 33 momenta with |n|^2 <= 3, all
    # Gamma pairs (A, A); projections and correlator timed after the step
    corr = None
    if len(loops) >= 2:
        mom = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
        mom += [(2, 0, 0), (0, 2, 0), (0, 0, 2), (-2, 0, 0), (0, -2, 0), (0, 0, -2)]
        neg = [(-a, -b, -c) for a, b, c in mom]
        L1 = torch.from_numpy(loops[0]).cuda()
        L2 = torch.from_numpy(loops[1]).cuda()
        lat.disconnected_corr(lat.momentum_project(L1, mom), lat.momentum_project(L2, neg),
                              [(g, g) for g in range(len(gam))])  # warm-up (allocations)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        P1 = lat.momentum_project(L1, mom)
        P2 = lat.momentum_project(L2, neg)
        tp = time.perf_counter()
        D = lat.disconnected_corr(P1, P2, [(g, g) for g in range(len(gam))])
        torch.cuda.synchronize()
        td = time.perf_counter()
        d0 = D[1, mom.index((0, 0, 0))].real.cpu().numpy()  # gamma_5 - gamma_5, p = 0
        # connected pseudoscalar function from a point source at the origin, local and
        # Gaussian-smeared (alpha 4, n 50, normalised per step by 1 + 6 alpha)
        prm = fl.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=solver)
        tq = time.perf_counter()
        c_loc = lat.pion_corr(0, prm, smear_source=False, smear_sink=False)[0].real
        tr = time.perf_counter()
        c_sm = lat.pion_corr(0, prm, 4.0, 50, 25.0, True, True)[0].real
        ts = time.perf_counter()
        corr = {"momenta": len(mom), "gamma_pairs": len(gam),
                "projection_us_per_loop_set": round((tp - tc) * 1e6 / 2, 1),
                "correlator_us": round((td - tp) * 1e6, 1),
                "D_g5g5_p0_t0_3": [float(x) for x in d0[:4]],
                "pion_corr_local_ms": round((tr - tq) * 1e3, 1),
                "pion_corr_smeared_ms": round((ts - tr) * 1e3, 1),
                "C_pi_local_t0_3": [float(x) for x in c_loc[:4]],
                "C_pi_smeared_t0_3": [float(x) for x in c_sm[:4]],
                "R_D_over_Cpi_local_t0_3": [float(d0[t] / c_loc[t]) for t in range(4)]}
        log(f"[bench] momentum projection {corr['projection_us_per_loop_set']} us per loop set, "
            f"correlator {corr['correlator_us']} us")

    if args.timed_only:
        print(json.dumps({"metric": METRIC, "value": round(value, 3), "unit": "solves/s", "steps": args.steps,
                          "hopping_kernel": {"launches": prof["launches"], "avg_launch_us": round(avg_us, 2),
                                             "achieved_GBs": round(achieved, 1)},
                          "end_hop_kernel": {"launches": profs["end_hop"]["launches"],
                                             "avg_launch_us": round(profs["end_hop"]["avg_us"], 2),
                                             "achieved_GBs": round(profs["end_hop"]["achieved"], 1)},
                          "vector_update_kernel": {"launches": profs["vector_update"]["launches"],
                                                   "avg_launch_us": round(profs["vector_update"]["avg_us"], 2),
                                                   "achieved_GBs": round(profs["vector_update"]["achieved"], 1)}}),
              flush=True)
        return
    # the other workloads of the path, timed once each outside the timed region:
    # exact loops of one whole timeslice, the uneven truncated-solver batch of
    # three lattices, and the gradient of exact loops
    extras = None
    if not args.no_extras:
        extras = {}
        gx = [0, 15]
        We = S.WORKLOADS["exact_8x8x8x16"]
        le = fl.Lattice(We["dims"], We["bc_t"], device=0)
        le.set_gauge(S.random_links(We["dims"], We["eps"], We["link_seed"]))
        le.set_kappa(We["kappa"])
        pe = fl.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=solver, batch=768)
        le.loops_exact([1], gam, pe)  # warm-up (one timeslice)
        torch.cuda.synchronize()
        w0 = time.monotonic_ns()
        t_e = time.perf_counter()
        le.loops_exact([0], gam, pe)
        torch.cuda.synchronize()
        t_e = time.perf_counter() - t_e
        window("exact_8x8x8x16_timeslice", w0)
        ns = 12 * We["dims"][0] * We["dims"][1] * We["dims"][2]
        extras["exact_loops_8x8x8x16_one_timeslice"] = {
            "point_sources": ns, "seconds": round(t_e, 3), "solves_per_s": round(ns / t_e, 1),
            "inner": f"{args.solver} {args.prec}, tol 1e-12", "gammas": len(gam)}
        log(f"[bench] exact loops 8^3x16, one timeslice: {ns} solves in {t_e:.2f} s ({ns / t_e:.0f} solves/s)")
        le.close()
        names = ["tsm_8x8x8x8", "tsm_12x12x12x24", "tsm_16x16x16x32"]
        lts = []
        for nme in names:
            Wt = S.WORKLOADS[nme]
            lt = fl.Lattice(Wt["dims"], Wt["bc_t"], device=0)
            lt.set_gauge(S.random_links(Wt["dims"], Wt["eps"], Wt["link_seed"]))
            lt.set_kappa(Wt["kappa"])
            lts.append((lt, Wt))
        qs = [fl.NoiseParams(noise=fl.NOISE_CZ2, seed=Wt["noise_seed"], r0=0, n_lp=64, n_hp=4, dilution=0,
                             t_begin=0, t_end=Wt["dims"][3]) for (_, Wt) in lts]
        lp_t = fl.SolverParams(tol=1e-3, truncated=True)
        hp_t = fl.SolverParams(tol=1e-12)
        fl.loops_stochastic_multi([lt for (lt, _) in lts], qs, gam, lp_t, hp_t)  # warm-up (allocations)
        torch.cuda.synchronize()
        w0 = time.monotonic_ns()
        t_t = time.perf_counter()
        fl.loops_stochastic_multi([lt for (lt, _) in lts], qs, gam, lp_t, hp_t)
        torch.cuda.synchronize()
        t_t = time.perf_counter() - t_t
        window("uneven_tsm_batch", w0)
        extras["uneven_tsm_batch_8^4_12^3x24_16^3x32"] = {
            "lp_solves": 3 * 64, "hp_solves": 3 * 4, "lp_tol": 1e-3, "hp_tol": 1e-12, "seconds": round(t_t, 3)}
        log(f"[bench] uneven TSM batch (3 lattices, 64 LP + 4 HP each): {t_t:.2f} s")
        for (lt, _) in lts:
            lt.close()
        Wg = S.WORKLOADS["grad_12x12x12x24"]
        lg = fl.Lattice(Wg["dims"], Wg["bc_t"], device=0)
        lg.set_gauge(S.random_links(Wg["dims"], Wg["eps"], Wg["link_seed"]))
        lg.set_kappa(Wg["kappa"])
        Vsg = Wg["dims"][0] * Wg["dims"][1] * Wg["dims"][2]
        wg = np.ones((len(gx), 1, Vsg), complex)
        torch.cuda.synchronize()
        t_g = time.perf_counter()
        lg.loops_grad([0], gx, wg, fl.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=solver,
                                                   batch=768))
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t_g
        extras["gradient_12x12x12x24_one_timeslice"] = {
            "point_sources": 12 * Vsg, "gammas": len(gx), "seconds": round(t_g, 3),
            "inner": f"{args.solver} {args.prec}, tol 1e-12 (forward solves; adjoints by g5-hermiticity)"}
        log(f"[bench] gradient 12^3x24, one timeslice ({12 * Vsg} sources): {t_g:.2f} s")
        lg.close()
        # the paper's solver (BiCGStab; the library's default: FP32 vectors and
        # links, FP64 reliable updates) on 96 diluted Z4 sources of the
        # benchmark's lattice (8 timeslices x 4 spins x 3 colours), for
        # comparison with the timed CGNR
        comps96 = [(t, sp, co) for t in range(1, dims[3], 4) for sp in range(4) for co in range(3)]
        b96 = torch.from_numpy(S.z4_diluted_sources(dims, comps96, W["noise_seed"] + 1)).to("cuda")
        pb = fl.SolverParams(tol=1e-12)
        lat.solve(b96, pb, check=False)  # warm-up (allocations)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        _, info_b = lat.solve(b96, pb, check=False)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t_b
        its_b = [i["iters"] for i in info_b]
        extras["bicgstab_fp32_16x16x16x32_96_sources"] = {
            "solves": len(info_b), "converged": int(sum(i["converged"] for i in info_b)),
            "seconds": round(t_b, 3), "solves_per_s": round(len(info_b) / t_b, 1),
            "iterations_mean": round(float(np.mean(its_b)), 1), "iterations_max": int(max(its_b)),
            "max_true_resid_full_operator": float(max(i["true_resid"] for i in info_b)),
            "inner": "bicgstab f32 (12-real links), tol 1e-12"}
        log(f"[bench] BiCGStab FP32 on 96 sources of 16^3x32: {t_b:.2f} s, {np.mean(its_b):.1f} iterations")
        del b96

    # accuracy and the plain FP64 single-RHS reference on sources of the same workload
    # the plain FP64 single-RHS GPU solve (the denominator of the batched
    # mixed-precision speed-up) on sources of the workload's shape: Z4 values
    # on one timeslice, spin and colour each (seeded numpy, the same arrays for
    # the GPU and for the oracle below)
    comps = [(0, 0, 0), (5, 1, 0), (17, 2, 0), (31, 3, 0)]
    nfp64 = max(1, args.fp64_rhs)
    b = S.z4_diluted_sources(dims, comps[:max(2, nfp64)], W["noise_seed"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(nfp64):
        x64, info64 = lat.solve(b[k:k + 1], fl.SolverParams(tol=1e-12, inner_prec=fl.PREC_F64, gauge_reals=18))
    torch.cuda.synchronize()
    fp64_rate = nfp64 / (time.perf_counter() - t1)
    x_mp, info_mp = lat.solve(b[:1], fl.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=solver))
    log(f"[bench] FP64 single-RHS GPU: {fp64_rate:.2f} solves/s ({info64[0]['iters']} iterations); "
        f"mixed: {info_mp[0]['iters']} iterations, {info_mp[0]['updates']} FP64 updates")

    cpu = None
    loop_err = None
    if not args.no_cpu_baseline:
        cpu, loop_err = cpu_baseline(U, b, x_mp, dims, bc, kappa, gam)

    Vh = S.volume(dims) // 2

    def hop_roof(name):
        # site x right-hand-side pairs per launch from the algorithmic bytes
        # (8 links per site once, the hop's fields once per pair); the FP32
        # rate counts the hopping term's flops only
        pr, fields, hop = profs[name], HOPS[name][1], HOPS[name][2]
        if args.solver != "cgnr":
            fields = {"first_hop": 2, "end_hop": 3, "vector_update": 7}[name]  # BiCGStab
        bpl = pr["bytes"] / max(1, pr["launches"])
        label = {"first_hop": "hopping term H_oe of Dhat p (no epilogue)",
                 "end_hop": "hopping term H_eo of Dhat^+ q with the fused update z -= alpha (q + c H q') "
                            "and |z|^2 (reads q and z at the site)" if args.solver == "cgnr" else
                            "hopping term H_eo of Dhat s with <t, s> and |t|^2 (reads s at the site)",
                 "vector_update": "vector update x += alpha p, p = z + beta p" if args.solver == "cgnr" else
                                  "vector update x += alpha p + omega s, r = s - omega t"}[name]
        # every kernel of the iteration is limited by the memory system; the
        # FP32 rate of the hopping term is reported beside a hop's figure
        out = {"kernel": f"{label}, {args.prec} storage" + (", 12-real links" if hop else "") +
                         ", iteration launches",
               "bound": "hbm", "achieved": round(pr["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(pr["achieved"] / HBM_PEAK_GBS, 4)}
        if hop:
            pairs = (bpl - 8 * LINK_BYTES[args.prec] * Vh) / (fields * SITE_BYTES[args.prec])
            tflops = FLOP_PER_SITE * pairs / (pr["avg_us"] * 1e-6) / 1e12 if pr["avg_us"] > 0 else 0.0
            out.update({"fp32_TFLOPs": round(tflops, 2), "fp32_frac": round(tflops / FP32_PEAK_TFLOPS, 4)})
        out.update({"traffic": profiled_traffic(args.prec, name), "avg_launch_us": round(pr["avg_us"], 2),
                    "launches": pr["launches"], "share_of_step": round(pr["ms"] * 1e-3 / T, 4),
                    "algorithmic_bytes_per_launch": round(bpl)})
        return out

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(T * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SU(3) links exp(i*0.6*H), Z4 noise; stands in for the 16^3x32 SESAM ensemble)",
        "config": {
            "workload": "stochastic loops, 16^3x32 lattice, eps=0.6, kappa=0.1596, Z4 noise, "
                        "spin-colour-time dilution, 384 diluted solves per step (one noise vector), "
                        "tol 1e-12 on the full operator, Gamma = 1, g5, g1..g4",
            "lattice": list(dims),
            "solves_per_step": solves_per_step,
            "inner": f"{args.solver} on the even-odd Schur system, " + {
                "f32": "fp32 vectors and 12-real links",
                "bf16": "fp32 vectors, bf16 12-real links",
                "h16": "16-bit fixed-point vectors (15-bit range, fp32 site scale) and 12-real links; hopping "
                       "term as exact int16 products summed in int32 (v_dot2_i32_i16), accumulated in fp32"}[args.prec]
                     + ", fp32 vector arithmetic, fp64 reliable updates",
            "batch": args.batch,
            "lds_mode": args.lds,
            "rt": args.rt,
            "group": args.group,
            "parallelism": "single GPU",
        },
        "roofline": hop_roof(dominant),
        "roofline_by_kernel": {name: hop_roof(name) for name in HOPS},
        "iteration_roofline": iteration_roofline(args.solver, args.prec, Vh, float(iters.sum()) / args.steps,
                                                 ITER_HOPS * float(iters.max()), T / args.steps),
        "cpu_baseline": cpu,
        "timed_solves": solves_summary,
        "fp64_single_rhs_gpu_solves_per_s": round(fp64_rate, 3),
        "speedup_vs_fp64_single_rhs": round(value / fp64_rate, 3),
        "loop_rel_err_vs_fp64": loop_err,
        "iterations": {"fp64_single": info64[0]["iters"], "mixed": info_mp[0]["iters"]},
        "disconnected_correlator": corr,
        "other_workloads": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
