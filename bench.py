"""Benchmark of the graph spectral filter hot path on one MI355X.

One step = one pass of the whole path over one noisy image of the workload:
build the BF operator (eq. (2), weights computed once), run CG for kmax_cg
steps (Algorithm 2) and block LOBPCG (m vectors, kmax_lob steps,
Algorithm 3).  Inputs are resident in HBM before timing starts.

value = pixel-vector-applies of the Laplacian per second over the whole step
(Mpixel-iters/s): per step, CG applies L_sym to 1 vector kmax_cg + 1 times and
LOBPCG applies it to m vectors kmax_lob + 1 times.

roofline: the dominant kernel (the stencil apply) timed with HIP events on its
own stream over `--roofline-reps` launches; achieved = algorithmic bytes per
launch / average duration, with algorithmic bytes per pixel
4 * ((K+1)/2 + 2m) for FP32 (each undirected edge once, the diagonal, x in, y
out; halo re-reads are not algorithmic).
cpu_baseline: the FP64 oracle (numpy/scipy, single thread) on a bounded crop
of the same image, in the same unit; also one such process per host core.
"""
from __future__ import annotations

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="image_1024_bf11")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--roofline-reps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serial", action="store_true", help="run CG and LOBPCG one after the other")
    ap.add_argument("--separate", action="store_true",
                    help="run CG and LOBPCG as two independent calls on two streams instead of the joint driver")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner measurement")
    ap.add_argument("--no-reguided", action="store_true", help="skip the re-guided (non-linear) filter measurement")
    ap.add_argument("--no-image-experiment", action="store_true",
                    help="skip the 5-point-lattice (diag L) image experiment (PSNR after 20 CG / LOBPCG steps)")
    ap.add_argument("--no-study-1d", action="store_true", help="skip the 1D filter study (Section 6)")
    ap.add_argument("--no-colour", action="store_true", help="skip the colour (CIE-Lab guidance) measurement")
    ap.add_argument("--no-gf", action="store_true", help="skip the GF apply measurement (4096^2, r = 8)")
    ap.add_argument("--no-1d", action="store_true", help="skip the 4096-sample 1D latency measurement")
    ap.add_argument("--no-4096", action="store_true",
                    help="skip the 4096^2 legs (BF 7x7 apply, precision study)")
    ap.add_argument("--oracle-side", type=int, default=160,
                    help="side of the image on which the precision study also runs the FP64 oracle")
    ap.add_argument("--learned-images", type=int, default=200, help="training images (10 pairs each)")
    ap.add_argument("--learned-eval", type=int, default=2048, help="side of the evaluation image")
    ap.add_argument("--precision-study", action="store_true",
                    help="only the precision study (the default run includes it): FP32 against all-FP64 LOBPCG "
                         "(m = 8, 100 steps) on the 4096^2 BF 7x7 and GF r = 8 workloads, and both against the "
                         "FP64 oracle on an --oracle-side image of the same class")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the stencil applies (m = 1 and m) and a 1 GiB copy, for hardware counters")
    return ap.parse_args()


def kernels_only(a):
    """Launch the dominant kernels alone, every tile choice of the BF apply
    (1, 2 and 4 rows per thread) for m = 1, the block width and the joint
    (m + 1)-column apply, 10 launches each, then a plain device copy of 1 GiB
    whose counter readings calibrate the byte counters."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    gsf.load_library()
    w = WORKLOADS[a.workload]
    shape, m = w["shape"], w["lobpcg_m"]
    n = int(np.prod(shape))
    prec = gsf.F32 if w["prec"] == "f32" else gsf.F64
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    _, noisy = make_signal(a.workload)
    x0 = torch.tensor(noisy.ravel(), dtype=dt, device="cuda")
    op = gsf.Operator(w["kind"], shape, x0, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"], prec)
    for mm in sorted({1, m}):
        xb = torch.randn((n, mm) if mm > 1 else (n,), dtype=dt, device="cuda")
        yb = torch.empty_like(xb)
        for rows in ((1, 2, 4) if w["kind"] == "bf" else (0,)):
            if rows:
                op.set_apply_rows(mm, rows)
            for _ in range(10):
                op.apply(xb, gsf.FORM_LSYM, out=yb)
    if w["kind"] == "bf":  # the joint (m + 1)-column apply of the joint CG + LOBPCG driver
        xb = torch.randn((n, m), dtype=dt, device="cuda")
        xc = torch.randn(n, dtype=dt, device="cuda")
        yb, yc = torch.empty_like(xb), torch.empty_like(xc)
        for rows in (1, 2, 4):
            op.set_apply_rows(m, rows)
            for _ in range(10):
                op.apply_joint(xb, xc, gsf.FORM_LSYM, out=yb, out2=yc)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernels_only": a.workload, "n": n, "copy_bytes": src.numel() * 4}), flush=True)


def _oracle_loop(args):
    """The oracle's CG(10) + LOBPCG(m, 5) on a crop, repeated for budget_s
    seconds after the operator build; returns (pixel-vector applies, seconds,
    build seconds).  One BLAS thread."""
    crop, radius, sigma_d, sigma_r, m, budget_s = args
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        op = oracle.build_operator("bf", crop, radius, sigma_d, sigma_r)
        t_build = time.perf_counter() - t0
        n = crop.size
        work = 0
        t0 = time.perf_counter()
        k_cg, k_lob = 10, 5
        while True:
            oracle.cg_filter(op, crop.ravel(), k_cg, data_prec="f32")
            oracle.lobpcg_filter(op, crop.ravel(), m, k_lob, data_prec="f32")
            work += n * ((k_cg + 1) + m * (k_lob + 1))
            if time.perf_counter() - t0 > budget_s:
                break
        return work, time.perf_counter() - t0, t_build


def cpu_baseline_all_cores(w, crop, budget_s):
    """The same loop in one process per available host core (at most 16),
    started together; the aggregate rate is the sum of the per-process
    rates."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    args = (crop, w["radius"], w["sigma_d"], w["sigma_r"], w["lobpcg_m"], budget_s)
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_loop, [args] * cores)
    rate = sum(r[0] / r[1] for r in res)
    return {"value": rate / 1e6, "unit": "Mpixel-iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} processes, each the single-thread loop on the same crop for {budget_s:.0f} s"}


def cpu_baseline(w, noisy, budget_s):
    """Time the oracle on a crop of the workload image: CG and LOBPCG steps,
    counted in the same unit (pixel-vector-applies per second), on one core
    and on every available core."""
    rows = max(32, min(noisy.shape[0], 128))
    crop = np.ascontiguousarray(noisy[:rows, :])
    k_cg, k_lob, m = 10, 5, w["lobpcg_m"]
    work, el, t_build = _oracle_loop((crop, w["radius"], w["sigma_d"], w["sigma_r"], m, budget_s))
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": work / el / 1e6, "unit": "Mpixel-iters/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model,
            "sample": f"{crop.shape[0]}x{crop.shape[1]} crop of the workload image, BF {2*w['radius']+1}x"
                      f"{2*w['radius']+1} operator (build {t_build:.1f} s excluded), repeated CG({k_cg}) + "
                      f"LOBPCG(m={m}, {k_lob}) for {el:.1f} s, FP64, single thread",
            "all_cores": cpu_baseline_all_cores(w, crop, min(10.0, budget_s)),
            "rows": rows_baseline()}


def rows_baseline():
    """The oracle timed on the workloads of the other measured rows (the
    image experiment, the 1D study, colour, re-guided), single thread, FP64:
    ms per run, on the whole workload or on the stated crop."""
    import oracle
    from synth import STUDY_1D, WORKLOADS, make_signal, study_signal
    out = {}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return round((time.perf_counter() - t0) * 1e3, 1)

    w = WORKLOADS["image_1024_cross5"]
    _, noisy = make_signal("image_1024_cross5")
    x = noisy.astype(np.float32).astype(np.float64)
    res = {"sample": "whole 1024x1024 image"}
    box = {}
    res["build_ms"] = timed(lambda: box.setdefault("op", oracle.build_operator(
        "bf", x, w["radius"], w["sigma_d"], w["sigma_r"], stencil=w["stencil"], norm=w["norm"])))
    op = box["op"]
    res["cg_ms"] = timed(lambda: oracle.cg_filter(op, x.ravel(), w["cg_iters"], data_prec="f32"))
    res["lobpcg_ms"] = timed(lambda: oracle.lobpcg_filter(op, x.ravel(), w["lobpcg_m"], w["lobpcg_iters"],
                                                          data_prec="f32"))
    out["image_experiment"] = res
    bf, gf, k = STUDY_1D["bf"], STUDY_1D["gf"], STUDY_1D["krylov_steps"]
    clean, noisy1 = study_signal(1000)
    opc = oracle.build_operator("bf", clean, bf["radius"], bf["sigma_d"], bf["sigma_r"])
    out["study_1d"] = {"sample": "N = 1000",
                       "bf_self_guided_ms": timed(lambda: oracle.power_filter_reguided(
                           "bf", noisy1, (1000,), bf["passes"], radius=bf["radius"], sigma_s=bf["sigma_d"],
                           sigma_r=bf["sigma_r"])),
                       "gf_self_guided_ms": timed(lambda: oracle.power_filter_reguided(
                           "gf", noisy1, (1000,), gf["passes"], radius=gf["radius"], eps=gf["eps"])),
                       "bf_cg_ms": timed(lambda: oracle.cg_filter(opc, noisy1, k))}
    w = WORKLOADS["image_1024_rgb_bf11"]
    _, rgb = make_signal("image_1024_rgb_bf11", shape=(128, 1024))
    lab = oracle.srgb_to_lab(rgb)
    box = {}
    res = {"sample": "128x1024 crop"}
    res["build_ms"] = timed(lambda: box.setdefault("op", oracle.build_operator(
        "bf", lab, w["radius"], w["sigma_d"], w["sigma_r"], channels=3)))
    res["cg_block_ms"] = timed(lambda: oracle.cg_filter_block(box["op"], rgb.reshape(-1, 3), w["cg_iters"]))
    out["colour"] = res
    w = WORKLOADS["image_1024_bf11"]
    _, g = make_signal("image_1024_bf11", shape=(128, 1024))
    out["reguided"] = {"sample": "128x1024 crop, 2 steps",
                       "cg_ms_per_step": round(timed(lambda: oracle.cg_filter_reguided(
                           "bf", g.ravel(), g.shape, 2, radius=w["radius"], sigma_s=w["sigma_d"],
                           sigma_r=w["sigma_r"])) / 2, 1)}
    return out


def batch_bench(seed=4):
    """Uneven batch (256 images with sides log-uniform in [64, 1024] and 64
    signals with lengths log-uniform in [2^10, 2^20], per-item BF/GF
    parameters, CG or LOBPCG(m=4), kmax 50, tol 1e-6): one graph launch of
    the batch against a sequential loop of single-item calls (operator build +
    solve per item, workspaces allocated beforehand, one stream)."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import batch_items, item_signal
    recipe = batch_items(seed=seed)
    items = []
    for it in recipe:
        _, noisy = item_signal(it)
        g = torch.tensor(noisy.ravel(), dtype=torch.float32, device="cuda")
        items.append(dict(kind=it["kind"], shape=it["shape"], radius=it["radius"], sigma_d=it["sigma_d"],
                          sigma_r=it["sigma_r"], eps=it["eps"], guidance=g, x0=g, method=it["method"], m=it["m"],
                          kmax=it["kmax"], tol=it["tol"]))
    npix = sum(int(np.prod(it["shape"])) for it in items)
    # the batch as recorded HIP graphs (one per branch stream, replayed by one
    # launch each) and the same batch issued from the host on every run
    # (the second takes the tiles the first tuned, as do the single-item calls)
    batch = gsf.Batch(items, prec=gsf.F32, autotune=True, graphs=True)
    batch_h = gsf.Batch(items, prec=gsf.F32, autotune=False, graphs=False)
    # sequential baseline: preallocated workspaces, one stream, no host syncs
    ops_ws, solver_ws, outs = [], [], []
    for it in items:
        op = gsf.Operator(it["kind"], it["shape"], it["guidance"], it["radius"], it["sigma_d"], it["sigma_r"],
                          it["eps"], gsf.F32)
        ops_ws.append(op.ws)
        solver_ws.append(op.workspace(gsf.METHOD_CG if it["method"] == "cg" else gsf.METHOD_LOBPCG, it["m"]))
        outs.append(torch.empty_like(it["x0"]))

    def sequential():
        keep = []
        for k, it in enumerate(items):
            op = gsf.Operator(it["kind"], it["shape"], it["guidance"], it["radius"], it["sigma_d"], it["sigma_r"],
                              it["eps"], gsf.F32, ws=ops_ws[k])
            if it["method"] == "cg":
                op.cg_filter(it["x0"], it["kmax"], tol=it["tol"], out=outs[k], ws=solver_ws[k], info=False)
            else:
                op.lobpcg_filter(it["x0"], it["m"], it["kmax"], tol=it["tol"], out=outs[k], ws=solver_ws[k],
                                 info=False)
            keep.append(op)
        return keep

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            del r
        return float(np.median(ts))

    sequential()
    t_seq = timed(sequential, 3)
    batch_h.run()
    t_host = timed(batch_h.run, 3)
    same_h = all(torch.equal(outs[k], it["out"]) for k, it in enumerate(items))
    batch.run()
    t_graph = timed(batch.run, 5)
    info = batch.info()
    same = same_h and all(torch.equal(outs[k], it["out"]) for k, it in enumerate(items))
    applies = sum(int(np.prod(it["shape"])) * (it["m"] if it["method"] == "lobpcg" else 1) * (info[k][0] + 1)
                  for k, it in enumerate(items))
    # the per-item convergence masks at work: the same batch with tol 1e-3,
    # where most items stop early and their remaining kernels return at once
    loose = [dict(it, tol=1e-3) for it in items]
    for it in loose:
        it.pop("out", None)
    batch_l = gsf.Batch(loose, prec=gsf.F32, autotune=False, graphs=True)
    batch_l.run()
    t_loose = timed(batch_l.run, 5)
    info_l = batch_l.info()
    return {"workload": "batch_256img_64sig", "items": len(items), "points": npix,
            "sequential_ms": round(t_seq * 1e3, 2), "batched_ms": round(t_graph * 1e3, 2),
            "host_issued_ms": round(t_host * 1e3, 2),
            "speedup": round(t_seq / t_graph, 3), "Mpixel_iters_per_s": round(applies / t_graph / 1e6, 1),
            "items_converged": int(sum(1 for i in info if i[1] == 0)), "outputs_equal_sequential": bool(same),
            "tol_1e-3": {"batched_ms": round(t_loose * 1e3, 2),
                         "items_converged": int(sum(1 for i in info_l if i[1] == 0)),
                         "mean_iters": round(float(np.mean([i[0] for i in info_l])), 1)}}


def learned_bench(n_images=200, side=512, eval_side=2048, tol=1e-6, kmax=20000, m=4, alpha=1e-2, inner=30,
                  snapshots=None):
    """Learned preconditioner: training pairs from the method itself on
    n_images noisy scenes of side^2 (BF 11x11, sigma_d = 2, sigma_r = 0.1,
    noise 0.05), 20 Adam epochs (batch 16, lr 1e-3), then block LOBPCG
    (m = 4, constraint, FP32 data, FP64 Rayleigh-Ritz) to a residual of tol on
    an unseen eval_side^2 scene: plain T = I, the learned T, and the T it is
    trained to imitate (`inner` CG steps on (L_sym + alpha I) y = r, the
    reference bound).  The learned run stops at three times the plain step
    count (beyond that it has lost).  Losses of the zero and the identity
    networks on the training pairs stand beside the trained one."""
    import torch
    import paper_1509_02468_amd as gsf
    from paper_1509_02468_amd import learned
    from synth import scene_2d, convnet_init

    snapshots = learned.SNAPSHOTS if snapshots is None else snapshots
    imgs = [scene_2d(side, side, 0.05, 5000 + i)[1] for i in range(n_images)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inputs, targets, cgi = learned.generate_pairs(imgs, 5, 2.0, 0.1, m=m, snapshots=snapshots, alpha=alpha)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    t0 = time.perf_counter()
    trainer, losses = learned.train(inputs, targets, side, side, convnet_init(5), epochs=20, batch=16, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pair_loss = {"trained": learned.dataset_loss(trainer.w.cpu().numpy(), inputs, targets, side, side),
                 "zero_net": learned.dataset_loss(np.zeros(gsf.NET_WEIGHTS, dtype=np.float32), inputs, targets,
                                                  side, side),
                 "identity_net": learned.dataset_loss(learned.identity_weights(), inputs, targets, side, side)}
    del inputs, targets
    g = scene_2d(eval_side, eval_side, 0.05, 5900)[1]
    gd = torch.tensor(g.ravel(), dtype=torch.float32, device="cuda")
    op = gsf.Operator("bf", (eval_side, eval_side), gd, 5, 2.0, 0.1, prec=gsf.F32)
    op.tune_apply(m)
    op.tune_apply(1)
    T = gsf.Precond(op, gd, trainer.wb)
    S = gsf.Precond.shifted(op, alpha, inner)
    ws = op.workspace(gsf.METHOD_LOBPCG, m)
    # one preconditioner application on an m-column block, device time
    R = torch.randn((op.n, m), dtype=torch.float32, device="cuda")
    Wout = torch.empty_like(R)
    T.apply(R, out=Wout)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(10):
        T.apply(R, out=Wout)
    ev[1].record()
    torch.cuda.synchronize()
    net_ms = ev[0].elapsed_time(ev[1]) / 10
    res = {}
    for name, P in (("plain", None), ("learned", T), ("shifted_solve", S)):
        cap = kmax if name != "learned" else max(3 * res["plain"]["iters"], 100)
        op.lobpcg_filter(gd, m, 3, constraint=True, ws=ws, precond=P)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = op.lobpcg_filter(gd, m, cap, tol=tol, constraint=True, ws=ws, precond=P)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"iters": info.iters, "ms": round(dt * 1e3, 1), "ms_per_iter": round(dt * 1e3 / max(info.iters, 1), 3),
                     "status": gsf.gsf.STATUS_NAMES.get(info.status, info.status), "kmax": cap,
                     "max_res": float(max(list(info.res)[:m])), "theta": [float(t) for t in list(info.theta)[:m]],
                     "fallbacks": info.fallbacks}
    net_flop = 2.0 * (16 * 2 * 9 + 16 * 16 * 9 + 16 * 9) * op.n * m
    return {"workload": f"learned_bf11_train{n_images}x{side}_eval{eval_side}",
            "train": {"pairs": n_images * len(snapshots), "snapshots": list(snapshots), "alpha": alpha,
                      "pair_gen_s": round(t_pairs, 1), "train_s": round(t_train, 1),
                      "cg_iters_mean": round(float(np.mean(cgi)), 1), "loss_first_epoch": round(float(losses[0]), 3),
                      "loss_last_epoch": round(float(losses[-1]), 3),
                      "loss_on_pairs": {k: round(v, 3) for k, v in pair_loss.items()}},
            "inference": {"ms_per_block": round(net_ms, 3), "m": m,
                          "tflops": round(net_flop / (net_ms * 1e-3) / 1e12, 1)},
            "tol": tol, "plain": res["plain"], "learned": res["learned"],
            "shifted_solve": dict(res["shifted_solve"], alpha=alpha, inner_cg_steps=inner),
            "iters_ratio_learned_over_plain": round(res["learned"]["iters"] / max(res["plain"]["iters"], 1), 3),
            "time_ratio_learned_over_plain": round(res["learned"]["ms"] / max(res["plain"]["ms"], 1e-9), 3),
            "iters_ratio_shifted_solve_over_plain": round(res["shifted_solve"]["iters"] / max(res["plain"]["iters"], 1),
                                                          3)}


def reguided_bench(steps=20, reps=3):
    """The re-guided (non-linear) filters on the metric's workload: every step
    takes the BF graph of the current iterate.  The passes evaluate the
    weights of eq. (2) where they use them (power: one pass per step; CG: a
    degree pass and the L pass), so no planes are stored.  Reports ms per
    step of CG and of the power filter, the weights evaluated per second by
    the power pass (n (K - 1) per step), and, for comparison, the operator
    build that stores the planes (what a rebuild per step would add)."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["image_1024_bf11"]
    shape = w["shape"]
    _, noisy = make_signal("image_1024_bf11")
    x0 = torch.tensor(noisy.ravel().astype(np.float32), device="cuda")
    par = dict(radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"])
    out = {"workload": "image_1024_bf11, graph rebuilt from the iterate every step", "steps": steps}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    for name, method in (("cg", gsf.METHOD_CG), ("power", gsf.METHOD_POWER)):
        ws = gsf.reguided_workspace("bf", shape, method, **par, prec=gsf.F32)
        y = torch.empty_like(x0)
        ms = timed(lambda: gsf.reguided_filter("bf", shape, x0, method, steps, **par, prec=gsf.F32, out=y, ws=ws,
                                               info=False))
        out[f"{name}_ms_per_step"] = round(ms / steps, 4)
        if method == gsf.METHOD_POWER:
            k = (2 * w["radius"] + 1) ** 2 - 1
            out["power_weights_per_s"] = float(f"{x0.numel() * k / (ms / steps * 1e-3):.4g}")
    op = gsf.Operator("bf", shape, x0, **par, prec=gsf.F32)
    ms = timed(lambda: [gsf.Operator("bf", shape, x0, **par, prec=gsf.F32, ws=op.ws) for _ in range(steps)])
    out["build_ms"] = round(ms / steps, 4)
    return out


def image_experiment_bench(reps=3, apply_reps=200):
    """The image experiment of Section 7 on its synthetic stand-in: 1024^2
    scene with noise variance 0.01, BF weights on the 5-point lattice
    (sigma_r = 0.1), (diag L) normalization, FP32.  Reports the PSNR of the
    noisy image and of 20 steps of CG and of LOBPCG (m = 1) with and without
    the constraint, the time of each run and of the build, and the 5-point
    apply (m = 1, L_sym form) against the HBM roofline: its algorithmic bytes
    per pixel are x, 1/sqrt(d), the two own weight planes and y (5 x 4 B; the
    mirrored weights and the neighbours' x come from cache)."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    name = "image_1024_cross5"
    w = WORKLOADS[name]
    shape = w["shape"]
    clean, noisy = make_signal(name)
    x0 = torch.tensor(noisy.ravel().astype(np.float32), device="cuda")
    par = dict(radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"], stencil=w["stencil"], norm=w["norm"])

    def psnr(y):
        y = y.double().cpu().numpy() if hasattr(y, "cpu") else np.asarray(y, dtype=np.float64)
        return round(float(10.0 * np.log10(1.0 / np.mean((y.ravel() - clean.ravel()) ** 2))), 3)

    def timed(fn, n=reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    op = gsf.Operator("bf", shape, x0, **par, prec=gsf.F32)
    out = {"workload": f"{name}: {shape[0]}x{shape[1]}, 5-point lattice, sigma_r={w['sigma_r']}, diag L "
                       f"normalization, FP32", "psnr_noisy": psnr(noisy)}
    out["build_ms"] = round(timed(lambda: gsf.Operator("bf", shape, x0, **par, prec=gsf.F32, ws=op.ws)), 4)
    k = w["cg_iters"]
    ws = op.workspace(gsf.METHOD_CG, 1)
    y = torch.empty_like(x0)
    out["cg_ms"] = round(timed(lambda: op.cg_filter(x0, k, out=y, ws=ws, info=False)), 4)
    out["psnr_cg"] = psnr(y)
    m, kl = w["lobpcg_m"], w["lobpcg_iters"]
    wsl = op.workspace(gsf.METHOD_LOBPCG, m)
    for c in (False, True):
        tag = "lobpcg_constraint" if c else "lobpcg"
        out[f"{tag}_ms"] = round(timed(lambda: op.lobpcg_filter(x0, m, kl, constraint=c, out=y, ws=wsl,
                                                                info=False)), 4)
        out[f"psnr_{tag}"] = psnr(y)
    out["iters"] = {"cg": k, "lobpcg": kl, "lobpcg_m": m}
    z = torch.empty_like(x0)
    ms = timed(lambda: [op.apply(x0, gsf.FORM_LSYM, out=z) for _ in range(apply_reps)], 3) / apply_reps
    algo = 5 * 4 * op.n
    out["apply"] = {"kernel": "bf_cross2d m=1 radius=1", "us_per_launch": round(ms * 1e3, 2),
                    "algorithmic_bytes_per_launch": algo,
                    "achieved_gbs": round(algo / (ms * 1e-3) / 1e9, 1),
                    "frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def gf_apply_bench(copy_gbs, reps=20):
    """The GF apply (Algorithm 1 on the fixed guidance, normalized) on the
    4096^2 GF workload (radius 8, FP32) for m = 1 and 8 columns, L_sym form,
    timed with HIP events on the launch stream over `reps` launches, against
    the HBM roofline.  Algorithmic bytes per point are what Algorithm 1 must
    move: x in and y out (4m each) and the guidance data g, mu_k and
    1/(sigma_k^2 + eps) once (12): 4(3 + 2m).  Anything else the kernels move
    (1/sqrt(d), intermediate window coefficients) is implementation traffic,
    measured by the counters (profiles/)."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["image_4096_gf8"]
    shape = w["shape"]
    n = int(np.prod(shape))
    _, noisy = make_signal("image_4096_gf8")
    g = torch.tensor(noisy.ravel().astype(np.float32), device="cuda")
    op = gsf.Operator("gf", shape, g, radius=w["radius"], eps=w["eps"], prec=gsf.F32)
    out = {"workload": f"image_4096_gf8 ({shape[0]}x{shape[1]}, GF r={w['radius']}, FP32), L_sym form",
           "copy_gbs": round(copy_gbs, 1)}
    s = torch.cuda.current_stream()
    for m in (1, 8):
        x = torch.rand((n, m) if m > 1 else (n,), device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        for _ in range(3):
            op.apply(x, gsf.FORM_LSYM, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            op.apply(x, gsf.FORM_LSYM, out=y)
        e1.record(s)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        algo = n * 4 * (3 + 2 * m)
        gbs = algo / (us * 1e-6) / 1e9
        out[f"m{m}"] = {"us_per_apply": round(us, 1), "algorithmic_bytes": algo, "achieved_gbs": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "frac_of_copy": round(gbs / copy_gbs, 4)}
    return out


def signal_1d_bench(reps=10):
    """The 4096-sample 1D workload (BF radius 5, sigma_d 3, sigma_r 0.2,
    FP64): microseconds per iteration of 30 power passes, 30 CG steps and 30
    LOBPCG (m = 3) steps, each run timed whole with HIP events (median of
    `reps`), issued eagerly and replayed from a HIP graph of the whole call.
    At 262 KB per apply this workload is bound by launch and reduction
    latency, not by bandwidth."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["signal_1d_4096"]
    _, noisy = make_signal("signal_1d_4096")
    x0 = torch.tensor(noisy, dtype=torch.float64, device="cuda")
    op = gsf.Operator("bf", w["shape"], x0, w["radius"], w["sigma_d"], w["sigma_r"], 0.0, gsf.F64)
    y = torch.empty_like(x0)
    wsp, wsc = op.workspace(gsf.METHOD_POWER), op.workspace(gsf.METHOD_CG)
    m = w["lobpcg_m"]
    wsl = op.workspace(gsf.METHOD_LOBPCG, m)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {"workload": "signal_1d_4096 (n = 4096, BF r = 5, FP64)"}
    for name, k, fn in (("power", w["power_iters"], lambda: op.power_filter(x0, w["power_iters"], out=y, ws=wsp)),
                        ("cg", w["cg_iters"], lambda: op.cg_filter(x0, w["cg_iters"], out=y, ws=wsc, info=False)),
                        ("lobpcg_m3", w["lobpcg_iters"],
                         lambda: op.lobpcg_filter(x0, m, w["lobpcg_iters"], out=y, ws=wsl, info=False)),
                        ("lobpcg_m3_constraint", w["lobpcg_iters"],
                         lambda: op.lobpcg_filter(x0, m, w["lobpcg_iters"], constraint=True, out=y, ws=wsl,
                                                  info=False))):
        ms = timed(fn)
        out[name] = {"iters": k, "ms": round(ms, 4), "us_per_iter": round(ms * 1e3 / k, 2)}
        # the same call recorded once into a HIP graph and replayed (no host
        # launches inside the timed region)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        ms_g = timed(graph.replay)
        out[name]["graph_us_per_iter"] = round(ms_g * 1e3 / k, 2)
        del graph
    return out


def image_4096_bf7_bench(copy_gbs, reps=20):
    """The 4096^2 BF 7x7 apply (sigma_d 2, sigma_r 0.15, FP32), where the
    working set (1.6 GB of weight planes) is far above the 256 MB
    Infinity Cache: m = 1 and m = 8 columns, L_sym form, tile tuned, timed
    with HIP events on the launch stream over `reps` launches.  Algorithmic
    bytes per point 4 ((K + 1)/2 + 2m) with K = 49."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["image_4096_bf7"]
    shape = w["shape"]
    n = int(np.prod(shape))
    _, noisy = make_signal("image_4096_bf7")
    g = torch.tensor(noisy.ravel().astype(np.float32), device="cuda")
    op = gsf.Operator("bf", shape, g, w["radius"], w["sigma_d"], w["sigma_r"], 0.0, gsf.F32)
    K = (2 * w["radius"] + 1) ** 2
    out = {"workload": f"image_4096_bf7 ({shape[0]}x{shape[1]}, BF {2 * w['radius'] + 1}x{2 * w['radius'] + 1}, "
                       f"FP32), L_sym form", "copy_gbs": round(copy_gbs, 1)}
    s = torch.cuda.current_stream()
    for m in (1, 8):
        x = torch.rand((n, m) if m > 1 else (n,), device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        best, times = op.tune_apply(m, reps=10)
        for _ in range(3):
            op.apply(x, gsf.FORM_LSYM, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            op.apply(x, gsf.FORM_LSYM, out=y)
        e1.record(s)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        algo = n * 4 * ((K + 1) // 2 + 2 * m)
        gbs = algo / (us * 1e-6) / 1e9
        out[f"m{m}"] = {"us_per_apply": round(us, 1), "rows_per_thread": best,
                        "us_by_rows_1_2_4": [round(t, 1) for t in times], "algorithmic_bytes": algo,
                        "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "frac_of_copy": round(gbs / copy_gbs, 4)}
        del x, y
    return out


def colour_bench(reps=3):
    """Colour guidance (Section 2: the photometric distance in CIE-Lab) on the
    1024^2 colour workload, FP32: the sRGB -> Lab conversion, the build from
    the 3-channel Lab guidance, and the three RGB channels filtered as one
    block (one 3-column apply per step) against three single-channel runs on
    the same operator; PSNR of the outputs."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal
    name = "image_1024_rgb_bf11"
    w = WORKLOADS[name]
    shape = w["shape"]
    clean, noisy = make_signal(name)
    xd = torch.tensor(noisy.reshape(-1, 3).astype(np.float32), device="cuda")
    cols = [xd[:, c].contiguous() for c in range(3)]
    par = dict(radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"], prec=gsf.F32, channels=3)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return round(float(np.median(ts)), 4)

    def psnr(y):
        y = y.double().cpu().numpy()
        return round(float(10.0 * np.log10(1.0 / np.mean((y.ravel() - clean.ravel()) ** 2))), 3)

    lab = torch.empty_like(xd)
    out = {"workload": f"{name}: {shape[0]}x{shape[1]} RGB, CIE-Lab guidance, BF {2 * w['radius'] + 1}x"
                       f"{2 * w['radius'] + 1}, sigma_r={w['sigma_r']} (Delta E), FP32",
           "psnr_noisy": round(float(10.0 * np.log10(1.0 / np.mean((noisy - clean) ** 2))), 3)}
    out["srgb_to_lab_ms"] = timed(lambda: gsf.srgb_to_lab(xd, out=lab))
    op = gsf.Operator("bf", shape, lab, **par)
    out["build_ms"] = timed(lambda: gsf.Operator("bf", shape, lab, **par, ws=op.ws))
    k, kp = w["cg_iters"], w["power_iters"]
    wsb = op.workspace(gsf.METHOD_CG, 3)
    ws1 = op.workspace(gsf.METHOD_CG, 1)
    y = torch.empty_like(xd)
    ys = [torch.empty_like(c) for c in cols]
    out["cg_block_ms"] = timed(lambda: op.cg_filter_block(xd, k, out=y, ws=wsb, info=False))
    out["psnr_cg"] = psnr(y)
    out["cg_3x_single_ms"] = timed(lambda: [op.cg_filter(cols[c], k, out=ys[c], ws=ws1, info=False)
                                            for c in range(3)])
    wpb = op.workspace(gsf.METHOD_POWER, 3)
    wp1 = op.workspace(gsf.METHOD_POWER, 1)
    out["power_block_ms"] = timed(lambda: op.power_filter_block(xd, kp, out=y, ws=wpb))
    out["psnr_power"] = psnr(y)
    out["power_3x_single_ms"] = timed(lambda: [op.power_filter(cols[c], kp, out=ys[c], ws=wp1) for c in range(3)])
    out["iters"] = {"cg": k, "power": kp}
    # the 3-column apply against the HBM roofline: 60 weight planes,
    # 1/sqrt(d), 3 values in and 3 out per point
    z = torch.empty_like(xd)
    napp = 100
    ms = timed(lambda: [op.apply(xd, gsf.FORM_LSYM, out=z) for _ in range(napp)]) / napp
    K = (2 * w["radius"] + 1) ** 2
    algo = 4 * ((K + 1) // 2 + 2 * 3) * xd.shape[0]
    out["apply"] = {"kernel": "bf_apply m=3", "us_per_launch": round(ms * 1e3, 2),
                    "algorithmic_bytes_per_launch": algo, "achieved_gbs": round(algo / (ms * 1e-3) / 1e9, 1),
                    "frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def study_1d_bench(reps=3):
    """The 1D filter study of Section 6 on both signal lengths, FP64: RMS
    error against the clean signal and run time of the self-guided BF (500
    re-guided passes), the self-guided GF (20 passes), BF-CG with the
    noiseless guidance (20 steps), and the GF-accelerated CG / LOBPCG and
    BF-LOBPCG (20 steps, noiseless guidance)."""
    import torch
    import paper_1509_02468_amd as gsf
    from synth import STUDY_1D, study_signal
    bf, gf, k = STUDY_1D["bf"], STUDY_1D["gf"], STUDY_1D["krylov_steps"]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return r, round(float(np.median(ts)), 3)

    out = {"workload": "G3 piecewise-linear signals, sigma 0.1; BF radius 1 (sigma_d 1, sigma_r 0.1), "
                       "GF radius 2 (eps 0.01); FP64", "passes": {"bf": bf["passes"], "gf": gf["passes"],
                                                                 "krylov": k}}
    for n in STUDY_1D["sizes"]:
        clean, noisy = study_signal(n)
        gd = torch.tensor(clean, device="cuda")
        xd = torch.tensor(noisy, device="cuda")

        def rms(y):
            return round(float(np.sqrt(np.mean((y.cpu().numpy() - clean) ** 2))), 5)
        res = {"noisy_rms": round(float(np.sqrt(np.mean((noisy - clean) ** 2))), 5)}
        y, ms = timed(lambda: gsf.reguided_filter("bf", (n,), xd, gsf.METHOD_POWER, bf["passes"],
                                                  radius=bf["radius"], sigma_d=bf["sigma_d"],
                                                  sigma_r=bf["sigma_r"], prec=gsf.F64, info=False)[0])
        res["bf_self_guided"] = {"rms": rms(y), "ms": ms}
        y, ms = timed(lambda: gsf.reguided_filter("gf", (n,), xd, gsf.METHOD_POWER, gf["passes"],
                                                  radius=gf["radius"], eps=gf["eps"], prec=gsf.F64, info=False)[0])
        res["gf_self_guided"] = {"rms": rms(y), "ms": ms}
        ops = {"bf": gsf.Operator("bf", (n,), gd, radius=bf["radius"], sigma_d=bf["sigma_d"],
                                  sigma_r=bf["sigma_r"], prec=gsf.F64),
               "gf": gsf.Operator("gf", (n,), gd, radius=gf["radius"], eps=gf["eps"], prec=gsf.F64)}
        for name, op in ops.items():
            y, ms = timed(lambda: op.cg_filter(xd, k, info=False)[0])
            res[f"{name}_cg"] = {"rms": rms(y), "ms": ms}
            y, ms = timed(lambda: op.lobpcg_filter(xd, 1, k, info=False)[0])
            res[f"{name}_lobpcg"] = {"rms": rms(y), "ms": ms}
        out[f"n{n}"] = res
    return out


def precision_study(oracle_side=160):
    """Per-result errors of the precision modes (the 4096^2 workloads, BF 7x7
    and GF radius 8, LOBPCG m = 8, 100 steps): FP32 data with MFMA Gram and
    FP64 Rayleigh-Ritz against the all-FP64 GPU run at 4096^2 (Ritz values,
    output, residuals, time per step), and both against the FP64 oracle at
    oracle_side^2 (same generator class and operators; the oracle cannot run
    at 4096^2 in bounded time)."""
    import torch
    import paper_1509_02468_amd as gsf
    import oracle
    from synth import WORKLOADS, make_signal, scene_2d

    def run(kind, shape, x, prec, w, m, k):
        dt = torch.float32 if prec == gsf.F32 else torch.float64
        xd = torch.tensor(x.ravel(), dtype=dt, device="cuda")
        op = gsf.Operator(kind, shape, xd, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"], prec)
        ws = op.workspace(gsf.METHOD_LOBPCG, m)
        op.lobpcg_filter(xd, m, 2, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y, info = op.lobpcg_filter(xd, m, k, ws=ws)
        torch.cuda.synchronize()
        return y.double().cpu().numpy(), np.array(list(info.theta)[:m]), np.array(list(info.res)[:m]), \
            time.perf_counter() - t0

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {}
    for name in ("image_4096_bf7", "image_4096_gf8"):
        w = WORKLOADS[name]
        m, k = w["lobpcg_m"], w["lobpcg_iters"]
        _, x = make_signal(name)
        x32 = x.astype(np.float32).astype(np.float64)
        y32, t32, r32, s32 = run(w["kind"], w["shape"], x32, gsf.F32, w, m, k)
        y64, t64, r64, s64 = run(w["kind"], w["shape"], x32, gsf.F64, w, m, k)
        res = {"full": {"shape": list(w["shape"]), "m": m, "steps": k,
                        "fp32_vs_fp64_theta_abs": float(np.abs(t32 - t64).max()),
                        "fp32_vs_fp64_theta_rel": float(np.abs(t32 / t64 - 1).max()),
                        "fp32_vs_fp64_y_rel": rel(y32, y64),
                        "fp32_res_max": float(r32.max()), "fp64_res_max": float(r64.max()),
                        "fp32_s": round(s32, 3), "fp64_s": round(s64, 3),
                        "fp32_ms_per_step": round(s32 * 1e3 / k, 3), "fp64_ms_per_step": round(s64 * 1e3 / k, 3)}}
        xs = scene_2d(oracle_side, oracle_side, w["sigma"], w["seed"])[1].astype(np.float32).astype(np.float64)
        shp = (oracle_side, oracle_side)
        ys32, ts32, _, _ = run(w["kind"], shp, xs, gsf.F32, w, m, k)
        ys64, ts64, _, _ = run(w["kind"], shp, xs, gsf.F64, w, m, k)
        ref = oracle.build_operator(w["kind"], xs, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"])
        t0 = time.perf_counter()
        yo, to, _, _ = oracle.lobpcg_filter(ref, xs.ravel(), m, k)
        res["oracle"] = {"shape": list(shp), "oracle_s": round(time.perf_counter() - t0, 1),
                         "fp64_theta_abs": float(np.abs(ts64 - to).max()), "fp64_y_rel": rel(ys64, yo),
                         "fp32_theta_abs": float(np.abs(ts32 - to).max()), "fp32_y_rel": rel(ys32, yo)}
        out[name] = res
    return out


def main():
    a = _args()
    if a.kernels_only:
        kernels_only(a)
        return
    if a.precision_study:
        import torch
        import paper_1509_02468_amd as gsf
        gsf.load_library()
        print(json.dumps({"precision_study": precision_study(a.oracle_side)}))
        return
    if a.gpus != 1:
        print(json.dumps({"error": f"--gpus {a.gpus}: the filters run on one GPU; there is no multi-GPU path (use --gpus 1)"}))
        sys.exit(2)
    import torch
    import paper_1509_02468_amd as gsf
    from synth import WORKLOADS, make_signal

    gsf.load_library()
    torch.cuda.set_device(0)
    w = WORKLOADS[a.workload]
    shape = w["shape"]
    n = int(np.prod(shape))
    prec = gsf.F32 if w["prec"] == "f32" else gsf.F64
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    _, noisy = make_signal(a.workload)
    x0 = torch.tensor(noisy.ravel(), dtype=dt, device="cuda")
    kcg, klob, m = w["cg_iters"], w["lobpcg_iters"], w["lobpcg_m"]
    stream = torch.cuda.current_stream()

    # allocate everything once; steps reuse the buffers
    op = gsf.Operator(w["kind"], shape, x0, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"], prec)
    # pick the apply tile height once (process-wide, reused by every step's operator)
    tuned = {}
    for mm in sorted({1, m}):
        best, times = op.tune_apply(mm, reps=20)
        tuned[f"m{mm}"] = {"rows_per_thread": best, "us_by_rows_1_2_4": [round(t, 1) for t in times]}
    ws_cg = op.workspace(gsf.METHOD_CG)
    ws_lob = op.workspace(gsf.METHOD_LOBPCG, m)
    ws_joint = op.joint_workspace(m)
    y_cg = torch.empty_like(x0)
    y_lob = torch.empty_like(x0)

    # CG and LOBPCG are independent filters of the same operator.  Default: the
    # joint driver, whose step k of both filters shares one stencil pass (the
    # CG vector as a fifth column of the LOBPCG block) and runs the CG update
    # and direction as extra workgroups of LOBPCG's one-workgroup
    # Rayleigh-Ritz launch and of its update launch.
    # --separate: two independent calls on two streams (LOBPCG, the longer
    # chain, enqueued first); --serial: one after the other.  (A GF operator's
    # apply uses the handle's scratch planes, so its filters stay on one
    # stream.)
    mode = "serial" if (a.serial or w["kind"] != "bf") else ("separate" if a.separate else "joint")
    concurrent = mode == "separate"
    s_cg, s_lob = torch.cuda.Stream(), torch.cuda.Stream()

    def step():
        op_s = gsf.Operator(w["kind"], shape, x0, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"], prec)
        if mode == "joint":
            op_s.joint_filter(x0, kcg, x0, m, klob, out_cg=y_cg, out_lob=y_lob, ws=ws_joint, info=False)
            return op_s
        if not concurrent:
            op_s.cg_filter(x0, kcg, out=y_cg, ws=ws_cg, info=False)
            op_s.lobpcg_filter(x0, m, klob, out=y_lob, ws=ws_lob, info=False)
            return op_s
        built = torch.cuda.Event()
        built.record(stream)
        s_cg.wait_event(built)
        s_lob.wait_event(built)
        op_s.lobpcg_filter(x0, m, klob, out=y_lob, ws=ws_lob, info=False, stream=s_lob)
        op_s.cg_filter(x0, kcg, out=y_cg, ws=ws_cg, info=False, stream=s_cg)
        stream.wait_stream(s_cg)
        stream.wait_stream(s_lob)
        return op_s

    keep = []
    for _ in range(a.warmup):
        keep.append(step())
    torch.cuda.synchronize()
    keep.clear()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        keep.append(step())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / a.steps * 1e3
    applies = n * ((kcg + 1) + m * (klob + 1))
    value = applies / (el / a.steps) / 1e6

    # dominant kernel: the stencil apply the step runs most (joint mode: the
    # (m + 1)-column joint apply; else the m = 1 or the m-column apply), timed
    # alone with events on its own stream
    K = (2 * w["radius"] + 1) ** len(shape)
    esz = 4 if prec == gsf.F32 else 8
    rl = {}
    s2 = torch.cuda.Stream()

    def time_launches(launch):
        with torch.cuda.stream(s2):
            for _ in range(5):
                launch()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s2)
            for _ in range(a.roofline_reps):
                launch()
            e1.record(s2)
        e1.synchronize()
        return e0.elapsed_time(e1) / a.roofline_reps

    for mm in (1, m):
        xb = torch.randn((n, mm) if mm > 1 else (n,), dtype=dt, device="cuda")
        yb = torch.empty_like(xb)
        t_ms = time_launches(lambda: op.apply(xb, gsf.FORM_LSYM, out=yb, stream=s2))
        rl[f"m{mm}"] = (esz * ((K + 1) // 2 + 2 * mm) * n, t_ms)
    if mode == "joint":
        xb = torch.randn((n, m), dtype=dt, device="cuda")
        xc = torch.randn(n, dtype=dt, device="cuda")
        yb, yc = torch.empty_like(xb), torch.empty_like(xc)
        t_ms = time_launches(lambda: op.apply_joint(xb, xc, gsf.FORM_LSYM, out=yb, out2=yc, stream=s2))
        rl[f"m{m}+1"] = (esz * ((K + 1) // 2 + 2 * (m + 1)) * n, t_ms)
        dom = f"m{m}+1"
        dom_rows = tuned[f"m{m}"]["rows_per_thread"]
    else:
        # the block apply moves more bytes per launch and runs as often as the m = 1 apply
        dom = f"m{m}" if rl[f"m{m}"][1] * (klob + 1) >= rl["m1"][1] * (kcg + 1) else "m1"
        dom_rows = tuned[dom]["rows_per_thread"]
    algo, t_ms = rl[dom]
    achieved = algo / (t_ms * 1e-3) / 1e9
    # what a plain device copy reaches (read + write of 1 GiB), the practical ceiling
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    c1.synchronize()
    copy_gbs = 2 * src.numel() * 4 / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del src, dst
    # HBM bytes per launch from the committed counter passes, for the tile the
    # tuner chose (null when no entry covers that kernel)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE)).get(f"{a.workload}:{dom}:rows{dom_rows}")
            traffic = tr.get("bytes_per_launch") if tr else None
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "kernel": f"bf_apply {dom} rows_per_thread={dom_rows}", "us_per_launch": round(t_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": algo,
                **{f"{k}_us": round(v[1] * 1e3, 2) for k, v in rl.items()}}

    batch = None if a.no_batch else batch_bench()
    learned_res = None if a.no_learned else learned_bench(a.learned_images, eval_side=a.learned_eval)
    reguided_res = None if a.no_reguided else reguided_bench()
    image_res = None if a.no_image_experiment else image_experiment_bench()
    study_res = None if a.no_study_1d else study_1d_bench()
    colour_res = None if a.no_colour else colour_bench()
    gf_res = None if a.no_gf else gf_apply_bench(copy_gbs)
    sig_res = None if a.no_1d else signal_1d_bench()
    bf7_res = None if a.no_4096 else image_4096_bf7_bench(copy_gbs)
    prec_res = None if a.no_4096 else precision_study(a.oracle_side)
    cpu = None if a.no_cpu else cpu_baseline(w, noisy, a.cpu_seconds)
    out = {"metric": "Mpixel-iters/s of Laplacian apply", "value": round(value, 1), "unit": "Mpixel-iters/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == gsf.F32 else "f64", "data": "synthetic",
           "config": {"workload": a.workload, "shape": list(shape), "operator": f"{w['kind']} r={w['radius']}",
                      "cg_iters": kcg, "lobpcg_iters": klob, "lobpcg_m": m, "parallelism": "single-gpu",
                      "apply_tuning": tuned, "cg_lobpcg_mode": mode},
           "roofline": roofline, "cpu_baseline": cpu, "batch": batch, "learned": learned_res,
           "reguided": reguided_res, "image_experiment": image_res,
           "study_1d": study_res, "colour": colour_res, "gf_apply": gf_res, "signal_1d_4096": sig_res,
           "image_4096_bf7": bf7_res, "precision_study": prec_res}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
