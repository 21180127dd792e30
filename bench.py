#!/usr/bin/env python
"""Benchmark of the two-site DMRG hot path on one MI355X.

Workload (default): the K=36, N=36, M=1024 chain molecule (integral seed
1003).  Setup, untimed: build the MPO, draw the random initial MPS, run
--presweeps full sweeps (default 2) so that the state has the sector
structure of a production sweep.  Then one more full sweep is timed (sweep
seconds), the center moves to the middle pair (17, 18) by exact SVD splits,
the middle-pair eigenproblem is solved from one start vector in FP64, FP32
and BF16 (mixed vs FP64), and the warm-up steps run.  A timed step is one complete two-site DMRG step at the middle bond:
blocking of the renormalized operators, Davidson with the sigma vector,
sector-wise SVD truncation to M, environment update and the next guess.
Steps alternate between the pairs (17, 18) forward and (18, 19) backward, so
every step works at the middle of the chain.

The metric value is the sigma-vector rate: model flops of all sigma calls in
the timed steps divided by their GPU time (HIP events on the library stream).
The same JSON line carries the measured sweep seconds, the mixed-precision
comparison, the roofline of the sigma kernel and the CPU oracle baseline.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA, TFLOP/s; bf16x3 does six BF16 products per product of the
# model, so its peak in model flops is a sixth of the BF16 one
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0 / 6}


def source_hash():
    """sha256 over the sources that decide the sigma launches (kernels and the
    task-list builder)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "engine.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1605_02611_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def recorded_traffic(prec, presweeps):
    """HBM bytes per sigma launch from the committed rocprofv3 counter summary,
    only while the sources are the ones the counters were taken on and the
    state is the recorded one (the traffic of a launch depends on the state's
    blocks, not on how many steps are timed); otherwise None."""
    try:
        txt = open(os.path.join(ROOT, "profiles", "hbm_traffic_sigma_k36_m1024_fp64.txt")).read()
    except OSError:
        return None
    rec = None
    for line in txt.splitlines():
        if line.startswith("machine-readable:"):
            rec = json.loads(line.split(":", 1)[1])
    if (rec is None or rec.get("sources_sha256") != source_hash() or prec != "fp64"
            or rec.get("presweeps", 0) != presweeps):
        return None
    return rec["traffic_bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(mps, j, budget_s):
    """The oracle's block-sparse sigma (oracle.blocksparse, FP64, NumPy) on a
    bounded sample of the benchmarked sigma: the middle pair of the K=36
    M=1024 workload with the sector structure of the benchmarked state,
    random environment operators and two-site vector, whole output sectors
    taken from the largest down until budget_s of oracle time is spent;
    rate = model flops of those sectors (oracle.flops) / oracle time."""
    from threadpoolctl import threadpool_info

    from oracle import blocksparse as ob
    from oracle import flops as of
    from oracle import mpo as omp
    from oracle.fermions import spin_orbital_integrals
    from tests import helpers as H
    from workloads import workload_integrals

    I = workload_integrals("chain_k36_m1024")
    K = I.h.shape[0]
    left = {(a, b): d for a, b, d in mps.bond(j)}
    right = {(a, b): d for a, b, d in mps.bond(j + 2)}
    t0 = time.time()
    ts, vs = spin_orbital_integrals(I.h, I.v)
    w = vs - vs.transpose(0, 1, 3, 2)
    Wj, Wj1 = omp._build_site(K, j, ts, w, vs), omp._build_site(K, j + 1, ts, w, vs)
    ch = [omp.channels(K, k) for k in (j, j + 1, j + 2)]
    rng = np.random.default_rng(0)
    trip = lambda d: [(q[0], q[1], m) for q, m in sorted(d.items())]
    shl = [omp.channel_qn(c) for c in ch[0]]
    shr = [omp.channel_qn(c) for c in ch[2]]
    nl = sum(r * c for bl in H.env_block_shapes(trip(left), shl) for _, _, r, c in bl)
    nr = sum(r * c for bl in H.env_block_shapes(trip(right), shr) for _, _, r, c in bl)
    L = H.env_values_to_blocks(rng.standard_normal(nl), trip(left), shl)
    R = H.env_values_to_blocks(rng.standard_normal(nr), trip(right), shr)
    mids = ob.middle_sectors(left, right)

    def rows_cols(q):
        r = sum(left.get((q[0] - a, q[1] - b), 0) for a, b in H.SITE_QN)
        c = sum(right.get((q[0] + a, q[1] + b), 0) for a, b in H.SITE_QN)
        return r * c
    psi = H.merged_blocks(rng.standard_normal(sum(rows_cols(q) for q in mids)), left, right)
    t_setup = time.time() - t0

    per = of.sigma_model_flops_by_sector(Wj, Wj1, ch[0], ch[1], ch[2], left, right)
    work = {q: float(sum(per.get(q, (0, 0)))) for q in mids}
    whole = sum(work.values())
    # sectors from the two-thirds quantile of work upwards, each taken only if the
    # rate measured so far says it fits the budget
    order = sorted(mids, key=lambda q: work[q])
    order = order[(2 * len(order)) // 3:]
    done, flops, dt = [], 0.0, 0.0
    for q in order:
        if done and dt + work[q] / (flops / max(dt, 1e-9)) > budget_s:
            break
        t1 = time.time()
        ob.sigma_sectors(Wj, Wj1, ch[0], ch[1], ch[2], left, right, L, R, psi, [q])
        dt += time.time() - t1
        done.append(q)
        flops += work[q]
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": ("oracle block-sparse sigma (FP64 NumPy, Eq. Hpartition per quantum-number block) at the "
                   "middle pair of the K=36 M=1024 workload with the benchmarked state's sectors, random "
                   "environments and vector: output sectors %s, %.3g of the %.3g model flops of one sigma, "
                   "in %.1f s; setup (MPO sites, random operators) %.1f s, not timed" % (
                       [list(q) for q in done], flops, whole, dt, t_setup)),
        "oracle_sigma_seconds_projected": dt * whole / flops,
    }


def full_sweeps(args, P, ctx, mpo, mps, prec, K, M, t_setup):
    """Full sweeps (forward and back over all pairs) from the random initial
    state; one JSON line with the energy and time of every sweep."""
    opts = P.default_opts(prec=prec, dav_tol=args.dav_tol, dav_max_iter=args.dav_iter,
                          refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
    rows = []
    for sw in range(args.sweeps):
        t1 = time.time()
        stats, _ = mps.sweep(M, 1, opts)
        st = stats[0]
        st["wall"] = time.time() - t1
        rows.append(st)
        log("sweep %d E %.10f %.1fs sigma %.1fs (%d calls, %.2f TFLOP/s) dav_iters %d disc %.2e" % (
            sw, st["energy"], st["wall"], st["sigma_seconds"], st["sigma_calls"],
            st["sigma_flops"] / max(st["sigma_seconds"], 1e-30) / 1e12, st["dav_iters"], st["discarded"]))
    e = mps.energy()
    fl = sum(r["sigma_flops"] for r in rows)
    ss = sum(r["sigma_seconds"] for r in rows)
    out = {"mode": "sweeps", "precision": args.prec, "K": K, "M": M, "n_sweeps": args.sweeps,
           "compress_tol": args.compress, "mpo_bond_dims": [int(d) for d in mpo.bond_dims()],
           "energy": e, "sweep_energies": [r["energy"] for r in rows],
           "sweep_seconds": [r["wall"] for r in rows], "sigma_tflops": fl / ss / 1e12,
           "sigma_seconds": ss, "sigma_calls": sum(r["sigma_calls"] for r in rows),
           "dav_iters": [r["dav_iters"] for r in rows], "discarded": [r["discarded"] for r in rows],
           "davidson_tol": args.dav_tol, "davidson_max_iter": args.dav_iter,
           "setup_seconds": time.time() - t_setup - sum(r["wall"] for r in rows)}
    print(json.dumps(out), flush=True)


def batched(args, P, torch):
    """The molecule batch: each instance swept alone in FP64 and in FP32, then
    all of them in lockstep with merged sigma launches (FP32)."""
    from workloads import batched_instances, chain_integrals, mps_values
    ctx = P.Context(0)
    n_sw = args.sweeps or 1
    inst = batched_instances(64)[:args.batched]
    mpos = []
    for K, M, seed in inst:
        I = chain_integrals(K, n_elec=K, seed=seed, rank=K)
        mpos.append(P.Mpo(ctx, I.h, I.v, K, K % 2))
    def fresh(b):
        K, M, seed = inst[b]
        return P.Mps.random(ctx, mpos[b], M, mps_values(seed, mpos[b].n_values(M)))
    res = {}
    for name, prec in (("seq_fp64", P.DMRG_FP64), ("seq_fp32", P.DMRG_FP32)):
        o = P.default_opts(prec=prec, dav_tol=args.dav_tol, dav_max_iter=args.dav_iter,
                           refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
        t0 = time.time()
        en = []
        for b in range(len(inst)):
            m = fresh(b)
            torch.cuda.synchronize()
            m.sweep(inst[b][1], n_sw, o)
            en.append(m.energy())
            del m
        res[name] = (time.time() - t0, en)
        log("%s %.1fs" % (name, res[name][0]))
    o = P.default_opts(prec=P.DMRG_FP32, dav_tol=args.dav_tol, dav_max_iter=args.dav_iter, refine_tol=1e-4)
    states = [fresh(b) for b in range(len(inst))]
    torch.cuda.synchronize()
    t0 = time.time()
    stats, bsig = P.sweep_batched(ctx, states, [x[1] for x in inst], n_sw, o)
    tb = time.time() - t0
    eb = [m.energy() for m in states]
    log("batched_fp32 %.1fs (batched sigma %.1fs)" % (tb, bsig))
    e64, e32 = np.array(res["seq_fp64"][1]), np.array(res["seq_fp32"][1])
    out = {"mode": "batched", "instances": len(inst), "sweeps": n_sw,
           "sizes": [[K, M] for K, M, _ in inst],
           "seconds": {"sequential_fp64": res["seq_fp64"][0], "sequential_fp32": res["seq_fp32"][0],
                       "batched_fp32": tb, "batched_sigma_wall": bsig},
           "speedup_vs_sequential_fp64": res["seq_fp64"][0] / tb,
           "speedup_vs_sequential_fp32": res["seq_fp32"][0] / tb,
           "max_abs_dE_batched_vs_sequential_fp32": float(np.abs(np.array(eb) - e32).max()),
           "max_abs_dE_batched_vs_sequential_fp64": float(np.abs(np.array(eb) - e64).max()),
           "energies_fp64": e64.tolist(), "energies_batched_fp32": eb,
           "davidson_tol": args.dav_tol, "davidson_max_iter": args.dav_iter}
    print(json.dumps(out), flush=True)


def precision_runs(P, mps, tol=1e-8, max_iter=60):
    """The same two-site eigenproblem (the current center) solved from the
    same start vector in every precision; the vector is restored after."""
    psi0 = mps.psi()
    rows = {}
    for name, prec, refine in (("fp64", P.DMRG_FP64, 0.0), ("fp32_refined", P.DMRG_FP32, 1e-4),
                               ("bf16_refined", P.DMRG_BF16, 1e-4), ("bf16x3_refined", P.DMRG_BF16X3, 1e-4),
                               ("fp32_only", P.DMRG_FP32, 0.0), ("bf16_only", P.DMRG_BF16, 0.0),
                               ("bf16x3_only", P.DMRG_BF16X3, 0.0)):
        mps.set_psi(psi0)
        o = P.default_opts(prec=prec, dav_tol=tol, dav_max_iter=max_iter, refine_tol=refine)
        t0 = time.time()
        th, rn, st = mps.solve(o)
        rows[name] = {"theta": th, "rnorm": rn, "converged": st["unconverged"] == 0, "iters": st["dav_iters"],
                      "sigma_calls": st["sigma_calls"], "sigma_seconds": st["sigma_seconds"],
                      "seconds": time.time() - t0,
                      "sigma_tflops": st["sigma_flops"] / max(st["sigma_seconds"], 1e-30) / 1e12}
        log("%-13s theta %.12f |r| %.2e iters %d sigma %.3fs" % (name, th, rn, st["dav_iters"], st["sigma_seconds"]))
    mps.set_psi(psi0)
    ref = rows["fp64"]["theta"]
    for r in rows.values():
        r["abs_dtheta_vs_fp64"] = abs(r["theta"] - ref)
        r["speedup_vs_fp64"] = rows["fp64"]["seconds"] / r["seconds"]
    return rows


def precision_check(args, P, mps, pre_e):
    """The same two-site eigenproblem (middle pair, state after the
    presweeps) solved from the same start vector in every precision."""
    rows = precision_runs(P, mps)
    print(json.dumps({"mode": "precision_check", "workload": "K=36 M=1024 middle pair after %d FP64 sweeps"
                      % args.presweeps, "presweep_energy": pre_e, "psi_elements": mps.psi_size(),
                      "davidson_tol": 1e-8, "davidson_max_iter": 60, "runs": rows}), flush=True)


def precision_sweeps(args, P, torch, mps, mpo, M, pre_e):
    """Mixed vs FP64 over whole sweeps: the state after the presweeps is
    saved, then swept args.precision_sweeps times in FP64, in FP32 and in
    BF16 (both refined in FP64 below a residual of 1e-4), every Davidson
    step converged to args.conv_tol (iteration cap args.conv_iter), each run
    from the saved state.  One JSON line: per run and sweep the energy,
    seconds, Davidson iterations and unconverged steps, |dE| against FP64."""
    import tempfile
    path = os.path.join(tempfile.mkdtemp(prefix="dmrg_state_"), "presweep.mps")
    mps.save(path)
    runs = {}
    for name, prec, refine in (("fp64", P.DMRG_FP64, 0.0), ("fp32_refined", P.DMRG_FP32, 1e-4),
                               ("bf16_refined", P.DMRG_BF16, 1e-4), ("bf16x3_refined", P.DMRG_BF16X3, 1e-4)):
        m = P.Mps.load(mps.ctx, mpo, path)
        o = P.default_opts(prec=prec, dav_tol=args.conv_tol, dav_max_iter=args.conv_iter, refine_tol=refine)
        rows = []
        for i in range(args.precision_sweeps):
            torch.cuda.synchronize()
            t1 = time.time()
            st, _ = m.sweep(M, 1, o)
            torch.cuda.synchronize()
            st = st[0]
            rows.append({"energy": st["energy"], "seconds": time.time() - t1, "sigma_seconds": st["sigma_seconds"],
                         "sigma_calls": st["sigma_calls"], "dav_iters": st["dav_iters"],
                         "unconverged_steps": st["unconverged"], "max_residual": st["max_residual"],
                         "discarded": st["discarded"]})
            log("%s sweep %d: E %.10f %.1fs iters %d unconverged %d max|r| %.1e" % (
                name, i, st["energy"], rows[-1]["seconds"], st["dav_iters"], st["unconverged"], st["max_residual"]))
        runs[name] = {"sweeps": rows, "energy": m.energy(), "seconds": sum(r["seconds"] for r in rows)}
        del m
    os.remove(path)
    ref = runs["fp64"]
    for r in runs.values():
        r["abs_dE_per_sweep_vs_fp64"] = [abs(a["energy"] - b["energy"]) for a, b in zip(r["sweeps"], ref["sweeps"])]
        r["abs_dE_vs_fp64"] = abs(r["energy"] - ref["energy"])
        r["within_1e-5"] = max(r["abs_dE_per_sweep_vs_fp64"]) <= 1e-5
        r["speedup_vs_fp64"] = ref["seconds"] / r["seconds"]
        r["all_steps_converged"] = all(x["unconverged_steps"] == 0 for x in r["sweeps"])
    print(json.dumps({"mode": "precision_sweeps",
                      "workload": "chain molecule K=36 N=36 M=%d, %d sweeps from the state after %d FP64 sweeps"
                                  % (M, args.precision_sweeps, args.presweeps),
                      "presweep_energy": pre_e, "davidson_tol": args.conv_tol, "davidson_max_iter": args.conv_iter,
                      "refine_below_residual": 1e-4, "tolerance_eh": 1e-5, "runs": runs}), flush=True)


def compress_study(args, P, torch):
    """Hamiltonian compression against the energy at converged states (Sec.
    "Hamiltonian compression"): the exact MPO is swept from the random state
    until the energy moves by less than 1e-9 Eh per sweep (at most 40
    sweeps, every Davidson step converged); for every threshold tau the
    converged exact state is evaluated with the compressed MPO (first order
    in the compression) and then swept with it to convergence (at most 12
    sweeps).  One JSON line: per tau the MPO bond dimensions, the converged
    energy, |E(tau) - E(0)|, the first-order shift and the last sweep's
    energy change."""
    import tempfile
    from workloads import WORKLOADS, workload_integrals, mps_values
    name = "chain_k20_m256"
    c = WORKLOADS[name]
    K, M = c["K"], c["M"]
    ctx = P.Context(0)
    I = workload_integrals(name)
    taus = [float(x) for x in args.compress_study.split(",")]
    if taus[0] != 0.0:
        taus = [0.0] + taus
    o = P.default_opts(dav_tol=args.conv_tol, dav_max_iter=args.conv_iter)
    path = os.path.join(tempfile.mkdtemp(prefix="dmrg_state_"), "exact.mps")
    rows = []
    for tau in taus:
        t0 = time.time()
        mpo = P.Mpo(ctx, I.h, I.v, I.n_elec, I.two_sz, compress_tol=tau)
        D = [int(d) for d in mpo.bond_dims()]
        row = {"tau": tau, "mpo_bond_dims": D, "D_mean": float(np.mean(D[1:K])), "D_max": max(D)}
        if tau == 0.0:
            m = P.Mps.random(ctx, mpo, M, mps_values(c["seed"], mpo.n_values(M)))
            max_sweeps = 40
        else:
            m = P.Mps.load(ctx, mpo, path)
            row["first_order_energy"] = m.energy()
            max_sweeps = 12
        es, conv = [], False
        for i in range(max_sweeps):
            st, _ = m.sweep(M, 1, o)
            es.append(st[0]["energy"])
            log("tau %g sweep %d E %.12f unconverged %d" % (tau, i, es[-1], st[0]["unconverged"]))
            if len(es) > 1 and abs(es[-1] - es[-2]) < 1e-9:
                conv = True
                break
        row.update({"energy": m.energy(), "sweeps": len(es), "converged": conv,
                    "last_sweep_change": abs(es[-1] - es[-2]) if len(es) > 1 else None,
                    "seconds": time.time() - t0})
        if tau == 0.0:
            m.save(path)
        rows.append(row)
        del m
    os.remove(path)
    e0 = rows[0]["energy"]
    for r in rows:
        r["abs_dE"] = abs(r["energy"] - e0)
        if "first_order_energy" in r:
            r["first_order_shift"] = r["first_order_energy"] - e0
        log("tau %-8g D_mean %7.1f D_max %5d E %.12f |dE| %.2e (%d sweeps)" % (
            r["tau"], r["D_mean"], r["D_max"], r["energy"], r["abs_dE"], r["sweeps"]))
    print(json.dumps({"mode": "compress_study", "workload": "%s: chain molecule K=%d N=%d M=%d" % (name, K, K, M),
                      "davidson_tol": args.conv_tol, "davidson_max_iter": args.conv_iter, "rows": rows}),
          flush=True)


def learned(args, P, torch):
    """Learned vs diagonal Davidson preconditioner: both runs start from the
    same random state; the learned run collects samples during the first
    sweeps (diagonal preconditioner), trains, then continues with the learned
    correction; the reference continues with the diagonal one."""
    from workloads import WORKLOADS, workload_integrals, mps_values
    name, n_col, n_cmp = args.learned.split(",")
    n_col, n_cmp = int(n_col), int(n_cmp)
    c = WORKLOADS[name]
    K, M = c["K"], c["M"]
    prec = {"fp64": P.DMRG_FP64, "fp32": P.DMRG_FP32, "bf16": P.DMRG_BF16, "bf16x3": P.DMRG_BF16X3}[args.prec]
    ctx = P.Context(0)
    I = workload_integrals(name)
    mpo = P.Mpo(ctx, I.h, I.v, I.n_elec, I.two_sz)
    vals = mps_values(c["seed"], mpo.n_values(M))
    net = P.Mlp(ctx, seed=7, capacity=1 << 22)
    kw = dict(prec=prec, dav_tol=args.dav_tol, dav_max_iter=args.dav_iter,
              refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
    out = {"mode": "learned", "workload": name, "K": K, "M": M, "precision": args.prec,
           "collect_sweeps": n_col, "compare_sweeps": n_cmp}
    runs = {}

    def sweeps(m, n, o, tag):  # one sweep at a time, a progress line each
        out = []
        for i in range(n):
            st, _ = m.sweep(M, 1, o)
            out.append(st[0])
            log("%s sweep %d: %.1fs E %.10f iters %d" % (tag, i, st[0]["seconds"], st[0]["energy"],
                                                        st[0]["dav_iters"]))
        return out

    modes = ("diagonal", "learned") if args.learned_mode == "both" else (args.learned_mode,)
    for mode in modes:
        m = P.Mps.random(ctx, mpo, M, vals)
        o = P.default_opts(collect=1 if mode == "learned" else 0, mlp=net if mode == "learned" else None, **kw)
        t0 = time.time()
        st = sweeps(m, n_col, o, mode + " (first sweeps)")
        log("%s: %d sweeps %.1fs E %.10f" % (mode, n_col, time.time() - t0, st[-1]["energy"]))
        if mode == "learned":
            t1 = time.time()
            ns = net.dataset(fetch=False)
            l0 = net.train(1, 4096, 1e-3, 11)
            loss = net.train(args.train_epochs, 4096, 1e-3, 12)
            out["training"] = {"samples": ns, "epochs": 1 + args.train_epochs, "loss_first_epoch": l0,
                               "loss_last_epoch": loss, "seconds": time.time() - t1}
            log("trained on %d samples: loss %.4f -> %.4f (%.1fs)" % (ns, l0, loss, out["training"]["seconds"]))
            o = P.default_opts(precond=1, mlp=net, **kw)
        t2 = time.time()
        st2 = sweeps(m, n_cmp, o, mode + " (compared sweeps)")
        runs[mode] = {"seconds": time.time() - t2, "sweep_seconds": [x["seconds"] for x in st2],
                      "dav_iters": [x["dav_iters"] for x in st2], "energies": [x["energy"] for x in st2],
                      "energy": m.energy(), "fallbacks": sum(x["precond_fallbacks"] for x in st2)}
        log("%s: compare sweeps %.1fs iters %s E %.10f" % (mode, runs[mode]["seconds"], runs[mode]["dav_iters"],
                                                           runs[mode]["energy"]))
        del m
    out["runs"] = runs
    if len(runs) == 2:
        out["iteration_ratio"] = sum(runs["learned"]["dav_iters"]) / max(1, sum(runs["diagonal"]["dav_iters"]))
        out["time_ratio"] = runs["learned"]["seconds"] / runs["diagonal"]["seconds"]
        out["abs_dE"] = abs(runs["learned"]["energy"] - runs["diagonal"]["energy"])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16", "bf16x3"])
    ap.add_argument("--dav-tol", type=float, default=1e-7)
    ap.add_argument("--dav-iter", type=int, default=24)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the timed full sweep (sweep seconds) after the presweeps")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the middle-pair FP64 / FP32 / BF16 eigenproblem comparison")
    ap.add_argument("--sweeps", type=int, default=0,
                    help="instead of middle steps: run this many full sweeps from the random "
                         "initial state and report energies and sweep seconds")
    ap.add_argument("--batched", type=int, default=0,
                    help="instead of middle steps: the first N instances of the 64-molecule batch "
                         "(K 12-24, M 128-512), --sweeps sweeps (default 1) sequential FP64, sequential "
                         "FP32 and batched FP32; energies and speedups")
    ap.add_argument("--learned", default="",
                    help="instead of middle steps: 'workload,collect,compare' e.g. 'chain_k24_m512,3,3': sweeps with the "
                         "diagonal preconditioner collecting training samples, training, then "
                         "`compare` sweeps learned vs diagonal from the same state")
    ap.add_argument("--precision-check", action="store_true",
                    help="instead of middle steps: after the presweeps, solve the middle two-site "
                         "problem from the same start vector in FP64, FP32 and BF16 (with and without "
                         "the FP64 refinement) and compare eigenvalues and sigma time")
    ap.add_argument("--precision-sweeps", type=int, default=0,
                    help="instead of middle steps: after the presweeps, this many full sweeps from "
                         "the same saved state in FP64, FP32 and BF16 (refined in FP64), every step "
                         "converged to --conv-tol; energies, |dE| against FP64 and time ratios")
    ap.add_argument("--compress-study", default="",
                    help="instead of middle steps: comma-separated MPO compression thresholds; the "
                         "K=20 M=256 chain swept to convergence with each (and the exact MPO)")
    ap.add_argument("--conv-tol", type=float, default=1e-6,
                    help="Davidson residual tolerance of --precision-sweeps")
    ap.add_argument("--conv-iter", type=int, default=400,
                    help="Davidson iteration cap of --precision-sweeps")
    ap.add_argument("--autotune", action="store_true",
                    help="run the launch autotuner at the middle pair before the timed steps")
    ap.add_argument("--compress", type=float, default=0.0,
                    help="MPO compression threshold (Hartree); 0 = exact MPO")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="oracle time budget of the CPU baseline sample")
    ap.add_argument("--train-epochs", type=int, default=30)
    ap.add_argument("--learned-mode", default="both", choices=["both", "diagonal", "learned"],
                    help="with --learned: run both preconditioners or only one (separate processes)")
    ap.add_argument("--presweeps", type=int, default=2,
                    help="untimed full sweeps from the random state before the timed middle steps")
    ap.add_argument("--calib", action="store_true",
                    help="run a 256 MiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1605_02611_amd as P
    from workloads import WORKLOADS, workload_integrals, mps_values

    prec = {"fp64": P.DMRG_FP64, "fp32": P.DMRG_FP32, "bf16": P.DMRG_BF16, "bf16x3": P.DMRG_BF16X3}[args.prec]
    if args.calib:
        src = torch.ones(32 << 20, device="cuda", dtype=torch.float64)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.batched:
        return batched(args, P, torch)
    if args.learned:
        return learned(args, P, torch)
    if args.compress_study:
        return compress_study(args, P, torch)
    c = WORKLOADS["chain_k36_m1024"]
    K, M = c["K"], c["M"]
    ctx = P.Context(0)
    t0 = time.time()
    I = workload_integrals("chain_k36_m1024")
    mpo = P.Mpo(ctx, I.h, I.v, I.n_elec, I.two_sz, compress_tol=args.compress)
    if args.compress:
        log("compressed MPO (tol %g, %.1fs): D %s" % (args.compress, time.time() - t0, list(mpo.bond_dims())))
    n = mpo.n_values(M)
    mps = P.Mps.random(ctx, mpo, M, mps_values(c["seed"], n))
    j = K // 2 - 1
    opts = P.default_opts(prec=prec, dav_tol=args.dav_tol, dav_max_iter=args.dav_iter,
                          refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
    pre_e = None
    if not args.sweeps and args.presweeps:
        # untimed: bring the random state close to the ground state first, so
        # that the timed steps see the sector structure of a production sweep
        for i in range(args.presweeps):  # one at a time, a progress line each
            st, _ = mps.sweep(M, 1, opts)
            pre_e = st[-1]["energy"]
            log("presweep %d: E %.10f (%.1fs)" % (i, pre_e, time.time() - t0))
    if args.precision_sweeps:
        return precision_sweeps(args, P, torch, mps, mpo, M, pre_e)
    sweep = None
    if not args.sweeps and not args.no_sweep and not args.precision_check:
        # sweep seconds: one full sweep (forward and back over every pair:
        # blocking, Davidson, SVD truncation, environment update), timed
        torch.cuda.synchronize()
        t2 = time.time()
        st, _ = mps.sweep(M, 1, opts)
        torch.cuda.synchronize()
        st = st[0]
        sweep = {"seconds": time.time() - t2, "energy": st["energy"], "sigma_seconds": st["sigma_seconds"],
                 "sigma_tflops": st["sigma_flops"] / max(st["sigma_seconds"], 1e-30) / 1e12,
                 "davidson_iterations": st["dav_iters"], "steps": st["n_steps"],
                 "unconverged_steps": st["unconverged"], "max_residual": st["max_residual"],
                 "discarded_weight": st["discarded"], "sweep_index": args.presweeps + 1}
        log("timed sweep: %.1fs E %.10f (%d of %d steps at the iteration cap)" % (
            sweep["seconds"], st["energy"], st["unconverged"], st["n_steps"]))
    for _ in range(0 if args.sweeps else j):
        mps.move(True)
    log("setup %.1fs: center %d, psi %d, D_mid %d" % (time.time() - t0, mps.center(), mps.psi_size(),
                                                      mpo.bond_dims()[j + 1]))
    if args.precision_check:
        return precision_check(args, P, mps, pre_e)
    mixed = None
    if not args.sweeps and not args.no_precision and args.prec == "fp64":
        # mixed vs FP64: the middle-pair eigenproblem in every precision from
        # the same start vector, each to the same residual tolerance
        t3 = time.time()
        rows = precision_runs(P, mps)
        mixed = {"workload": "middle pair (17, 18) after %d sweeps, same start vector" % (
                     args.presweeps + (sweep is not None)),
                 "davidson_tol": 1e-8, "davidson_max_iter": 60, "tolerance_eh": 1e-5,
                 "runs": rows,
                 "fp32_refined_within_1e-5": rows["fp32_refined"]["abs_dtheta_vs_fp64"] <= 1e-5,
                 "bf16_refined_within_1e-5": rows["bf16_refined"]["abs_dtheta_vs_fp64"] <= 1e-5,
                 "bf16x3_refined_within_1e-5": rows["bf16x3_refined"]["abs_dtheta_vs_fp64"] <= 1e-5,
                 "seconds": time.time() - t3}
    tuned = None
    if args.autotune:
        t3 = time.time()
        rep = P.autotune(ctx, mps, prec, reps=3)
        tuned = rep["best"]
        for c in sorted(rep["candidates"], key=lambda c: c["ms"]):
            log("autotune %s tiles %d/%d pieces %6d variant %d: %.3f ms" % (rep["key"], c["tile1"], c["tile2"],
                                                                             c["pieces"], c["variant"], c["ms"]))
        log("autotune %.1fs" % (time.time() - t3))
    if args.sweeps:
        return full_sweeps(args, P, ctx, mpo, mps, prec, K, M, t0)
    fwd = True
    for w in range(args.warmup):
        th, st = mps.step(M, fwd, opts)
        log("warmup %d theta %.10f" % (w, th))
        fwd = not fwd
    torch.cuda.synchronize()
    tot = dict(flops=0.0, sig=0.0, gemm=0.0, launches=0, calls=0, iters=0, unconverged=0)
    thetas = []
    t1 = time.time()
    for s in range(args.steps):
        th, st = mps.step(M, fwd, opts)
        fwd = not fwd
        thetas.append(th)
        tot["flops"] += st["sigma_flops"]
        tot["sig"] += st["sigma_seconds"]
        tot["gemm"] += st["gemm_seconds"]
        tot["launches"] += st["gemm_launches"]
        tot["calls"] += st["sigma_calls"]
        tot["iters"] += st["dav_iters"]
        tot["unconverged"] += st["unconverged"]
        log("step %d %s theta %.10f %.2fs sigma %d calls %.3fs" % (s, "fwd" if not fwd else "bwd", th,
                                                                  st["seconds"], st["sigma_calls"],
                                                                  st["sigma_seconds"]))
    torch.cuda.synchronize()
    wall = time.time() - t1
    sigma_tflops = tot["flops"] / tot["sig"] / 1e12
    gemm_tflops = tot["flops"] / tot["gemm"] / 1e12
    out = {
        "metric": "sigma-vector TFLOP/s + sweep seconds (K=36,M=1024); mixed vs FP64 at 1e-5 Eh",
        "value": sigma_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16-in/f32-acc", "bf16x3": "bf16x3-in/f32-acc"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "chain molecule K=36 N=36 2Sz=0 M=1024 (integral seed 1003), "
                               "two-site steps at the middle bond after %d sweeps from the random state%s" % (
                                   args.presweeps + (sweep is not None),
                                   " (the last one timed for sweep_seconds)" if sweep else ""),
                   "K": K, "M": M, "D_mid": int(mpo.bond_dims()[j + 1]), "psi_elements": mps.psi_size(),
                   "presweeps": args.presweeps, "presweep_energy": pre_e, "autotuned": tuned,
                   "davidson_tol": args.dav_tol, "davidson_max_iter": args.dav_iter,
                   "precision": args.prec, "mpo_compress_tol": args.compress},
        "sigma_calls": tot["calls"],
        "sigma_model_flops": tot["flops"],
        "step_tflops_wall": tot["flops"] / wall / 1e12,
        "thetas": thetas,
        "roofline": {"bound": "mfma", "achieved": gemm_tflops, "peak": PEAK[args.prec],
                     "unit": "TFLOP/s", "frac": gemm_tflops / PEAK[args.prec],
                     "traffic": (None if args.compress else
                                 recorded_traffic(args.prec, args.presweeps + (sweep is not None))),
                     "kernel": "lean_gemm<%d,1,*> (both sigma passes)" % prec,
                     "avg_launch_ms": tot["gemm"] / max(1, tot["launches"]) * 1e3,
                     "model_flops_per_launch": tot["flops"] / max(1, tot["launches"])},
        "sweep_seconds": sweep["seconds"] if sweep else None,
        "sweep": sweep,
        "mixed_vs_fp64": mixed,
        "unconverged_steps": tot["unconverged"],
    }
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(mps, j, args.cpu_seconds)
        except Exception as e:  # report, do not hide
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
