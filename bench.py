#!/usr/bin/env python3
"""Throughput of the Flow Fields hot path on one MI355X.

One step = one ff_flow_fields call on a 1024x436 synthetic pair (the
Sintel-sized plain workload: 16-channel uint8 descriptors, 7x7 SAD patch,
5 scales, 6 propagation steps per scale): descriptors of both images at every
scale, forward and backward fields, both consistency masks.  Inputs are
resident in device memory before the timed region.  Prints one JSON line.
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

METRIC = "Mpixel/s fwd+bwd Flow Field at 1024×436 (plain vs learned); EPE on synthetic GT"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_pair_seconds(pair, c, threads, min_seconds, max_runs=20):
    """Seconds per whole pair of the oracle on `threads` host threads,
    repeated until about min_seconds of work (at least one run)."""
    import oracle
    runs, t0 = 0, time.perf_counter()
    while runs < max_runs and (runs == 0 or time.perf_counter() - t0 < min_seconds):
        oracle.flow_fields(pair.img1, pair.img2, c.levels, c.iters, c.radius, c.R_num, c.R_den, c.eps, c.seed,
                           nthreads=threads)
        runs += 1
    return (time.perf_counter() - t0) / runs, runs


def cpu_baseline(pair, c, threads):
    """The oracle on the host cores: the whole 1024x436 pair (descriptors,
    fwd+bwd fields, consistency) on `threads` threads for about 10 s, and
    one run on a single thread."""
    H, W = pair.img1.shape
    s_nt, runs_nt = oracle_pair_seconds(pair, c, threads, 10.0)
    s_1t, _ = oracle_pair_seconds(pair, c, 1, 0.0, max_runs=1)
    return {"value": round(W * H / s_nt / 1e6, 4), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"{runs_nt} runs of one full {W}x{H} pair (descriptors, fwd+bwd fields, consistency) on "
                      f"{threads} threads, {s_nt * runs_nt:.2f} s in total; one run on 1 thread",
            "ms_per_pair": round(s_nt * 1e3, 1),
            "single_thread": {"value": round(W * H / s_1t / 1e6, 5), "ms_per_pair": round(s_1t * 1e3, 1)},
            "host_logical_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def config_legs(ff, torch, threads, reps=20):
    """The other single-pair workloads, GPU beside the oracle: 160x120
    (3 scales x 4 steps) and 1242x375 radial expansion (5 scales x 6 steps,
    R = 3/2); GPU ms per pair with HIP events (launch tables cached for the
    frame size, else the built-in ones), oracle ms on `threads` host threads
    (and one thread for the small pair)."""
    import dataclasses

    from ffgen import CONFIG_PARAMS, make_pair
    from paper_1703_02563_amd import autotune
    out = {}
    for cfg in (1, 3):
        p, c = make_pair(cfg), CONFIG_PARAMS[cfg]
        H, W = p.img1.shape
        prm = ff.Params(levels=c.levels, iters=c.iters, radius=c.radius, R_num=c.R_num, R_den=c.R_den, eps=c.eps,
                        seed=c.seed)
        tab = autotune.load(W, H, prm)  # this frame size's cached tables, else the built-in ones
        if tab is not None:
            prm = dataclasses.replace(prm, tuning=tab)
        i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
        runner = ff.FlowFields(W, H, prm, device=i1.device)
        for _ in range(3):
            runner(i1, i2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            runner(i1, i2)
        e1.record()
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / reps
        s_nt, _ = oracle_pair_seconds(p, c, threads, 2.0)
        leg = {"W": W, "H": H, "levels": c.levels, "iters": c.iters, "R": f"{c.R_num}/{c.R_den}",
               "gpu_ms_per_pair": round(gms, 4), "gpu_mpix_per_s": round(W * H / gms / 1e3, 2),
               "oracle_ms_per_pair": round(s_nt * 1e3, 1), "oracle_threads": threads,
               "n_evals": [int(v) for v in runner.out["n_evals"].cpu()]}
        if cfg == 1:
            s_1t, _ = oracle_pair_seconds(p, c, 1, 1.0)
            leg["oracle_1thread_ms_per_pair"] = round(s_1t * 1e3, 1)
        out[f"{W}x{H}"] = leg
    return out


# Integer-VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# 32-bit op (v_sad_u8: four byte |a-b| plus accumulate) per lane per clock.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
SAD_OPS_PER_EVAL = 7 * 7 * 16 // 4  # 784 byte differences = 196 v_sad_u8 per patch evaluation


# HBM traffic per launch of the scale-1 level kernel (both directions of the
# 1024x436 pair, as ff_flow_fields and the roofline leg launch it) from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE;
# profiles/level_kernel_traffic_1024x436.md), scaled by what the same
# counters read for a 256 MiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x
# 1.0).  Valid only for the kernel sources it was measured on.
TRAFFIC_BYTES = 20606.3 * 1024 * 2.0 + 6998.2 * 1024 * 1.0
TRAFFIC_SOURCES_SHA = "7ee290fff2ddf513"
TRAFFIC_VARIANT, TRAFFIC_PASSES = 31, 3  # scale-1 launch table the counters were taken with
# Vector-L1 tag accesses of 64 bytes per launch of the same kernel
# (TCP_TOTAL_CACHE_ACCESSES_sum, same run conditions; the L1 data path moves
# 64 bytes per clock per CU).
L1_ACCESSES = 26903544.8
L1_PEAK_TBPS = 256 * 64 * 2.4e9 / 1e12
# Matrix-core and VALU issue utilisation of the NN seed kernel (k_nn, both
# directions) from SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU and
# GRBM_GUI_ACTIVE (profiles/level_kernel_sq_1024x436.md); valid for the
# ff_nn.hip it was measured on.
NN_COUNTERS = {"mfma_busy": 0.185, "valu_issue": 0.740, "mfma_instructions": 1562624}
NN_SOURCES_SHA = "3b4b65b8af50d83f"
LEVEL_SOURCES = ("paper_1703_02563_amd/csrc/ff_level.hip", "paper_1703_02563_amd/csrc/ff_level_kernels.h",
                 "paper_1703_02563_amd/csrc/ff_level_s0.hip", "paper_1703_02563_amd/csrc/ff_device.h",
                 "paper_1703_02563_amd/csrc/ff_internal.h")


def level_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in LEVEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def roofline_level0(ff, torch, img1, img2, params, reps):
    """Times the scale-1 level kernel as ff_flow_fields launches it: both
    directions in one set of launches (ff_run_level_pair from the scale-2
    states), HIP events on the current stream, averaged per launch.
    Algorithmic work = the evaluations the launches compute for the cells
    they own (the kernel's work counter; evaluations that a consistent state
    makes unnecessary and recomputed halo cells are not counted) x 196
    v_sad_u8 lane-ops."""
    H, W = img1.shape
    L = params.levels
    ma = [ff.descriptors(img1, 1 << lv, wform=True) for lv in range(L)]
    mb = [ff.descriptors(img2, 1 << lv, wform=True) for lv in range(L)]
    Da, Wa = [m[1] for m in ma], [m[2] for m in ma]
    Db, Wb = [m[1] for m in mb], [m[2] for m in mb]
    Da1 = ff.descriptors(img1, 1, rowmajor=True)[2]
    Db1 = ff.descriptors(img2, 1, rowmajor=True)[2]
    keys = [ff.init_nn(Da1, Db1, Da[L - 1], Db[L - 1], 1 << (L - 1))[2],
            ff.init_nn(Db1, Da1, Db[L - 1], Da[L - 1], 1 << (L - 1))[2]]
    dev = img1.device
    prev = None
    for lv in range(L - 1, 0, -1):
        Wn, Hn = -(-W // (1 << lv)), -(-H // (1 << lv))
        fl = [torch.empty((Hn, Wn, 2), dtype=torch.int16, device=dev) for _ in range(2)]
        co = [torch.empty((Hn, Wn), dtype=torch.int32, device=dev) for _ in range(2)]
        if prev is None:
            ff.run_level_pair(Da[lv], Db[lv], lv, params, 1, fl, co, nn_keys=keys, wform_a=Wa[lv], wform_b=Wb[lv])
        else:
            ff.run_level_pair(Da[lv], Db[lv], lv, params, 2, fl, co, coarse_flows=prev[0], coarse_costs=prev[1],
                              wform_a=Wa[lv], wform_b=Wb[lv])
        prev = (fl, co)
    fl0 = [torch.empty((H, W, 2), dtype=torch.int16, device=dev) for _ in range(2)]
    co0 = [torch.empty((H, W), dtype=torch.int32, device=dev) for _ in range(2)]
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    work = torch.zeros(2, dtype=torch.int64, device=dev)
    scratch = torch.empty(2 * int(ff.lib().ff_run_level_scratch_bytes(W, H, 0)), dtype=torch.uint8, device=dev)

    def launch(counter=None, wk=None):
        ff.run_level_pair(Da[0], Db[0], 0, params, 2, fl0, co0, coarse_flows=prev[0], coarse_costs=prev[1],
                          n_evals=counter, n_work=wk, scratch=scratch, wform_a=Wa[0], wform_b=Wb[0])

    for _ in range(3):
        launch()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:  # timed without the counters
        a.record()
        launch()
        b.record()
    torch.cuda.synchronize()
    launch(cnt, work)  # the same call once more, counted (the counts do not vary between calls)
    torch.cuda.synchronize()
    # one call = `launches` launches of the scale-1 level kernel
    launches = ff.level_launches(params, 0)
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps / launches
    evals = int(cnt.sum().item()) / launches
    w_owned, w_all = (int(v) / launches for v in work.cpu())
    achieved = w_owned * SAD_OPS_PER_EVAL / (ms * 1e-3) / 1e12
    tun = params.tuning or ff.default_tuning()
    traffic = l1 = None
    if level_sources_sha() == TRAFFIC_SOURCES_SHA and tun.variant[0] == TRAFFIC_VARIANT \
            and tun.passes[0] == TRAFFIC_PASSES:
        traffic = round(TRAFFIC_BYTES)
        l1_tbps = L1_ACCESSES * 64 / (ms * 1e-3) / 1e12
        l1 = {"bytes_per_launch": round(L1_ACCESSES * 64), "achieved_TBps": round(l1_tbps, 3),
              "peak_TBps": round(L1_PEAK_TBPS, 2), "frac": round(l1_tbps / L1_PEAK_TBPS, 4)}
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "T int-op/s", "frac": round(achieved / VALU_PEAK_TOPS, 5), "traffic": traffic,
            "vector_l1": l1,
            "kernel": f"k_level<0,*> (scale 1, both directions per launch as in ff_flow_fields; "
                      f"{launches} launches per call, averages per launch)",
            "avg_launch_ms": round(ms, 5), "evals_per_launch": evals,
            "computed_owned_per_launch": w_owned, "computed_all_per_launch": w_all,
            "algorithmic_ops_per_launch": w_owned * SAD_OPS_PER_EVAL}


def nn_counters():
    """The NN seed kernel's counter figures, or None once ff_nn.hip has
    changed since they were taken."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1703_02563_amd/csrc/ff_nn.hip"), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    if sha != NN_SOURCES_SHA:
        return None
    return dict(NN_COUNTERS, kernel="k_nn (both directions)", source="profiles/level_kernel_sq_1024x436.md")


def batched_throughput(ff, torch, reps):
    """64 pairs of uneven sizes (256-1280 x 192-512, 12 polygon layers, t in
    +-100 px) in one ff_flow_fields_batched call, replayed from a HIP graph."""
    from ffgen import CONFIG_PARAMS, batch_shapes, make_pair
    from paper_1703_02563_amd.batch import BatchFlowFields
    c = CONFIG_PARAMS[4]
    shapes = batch_shapes()
    prm = ff.Params(levels=c.levels, iters=c.iters, radius=c.radius, R_num=c.R_num, R_den=c.R_den, eps=c.eps,
                    seed=c.seed)
    import dataclasses

    from paper_1703_02563_amd import autotune
    tables = autotune.load_batch(len(shapes), prm)
    log(f"bench: batch launch tables {tables if tables else '(built-in)'}")
    b = BatchFlowFields(shapes, dataclasses.replace(prm, tuning=tables))
    for k, shp in enumerate(shapes):
        p = make_pair(4, k, shape=shp)
        b.set_pair(k, torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda())
    b.capture()
    for _ in range(2):
        b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    mpix = sum(h * w for h, w in shapes) / 1e6
    return {"pairs": len(shapes), "mpix": round(mpix, 3), "ms_per_batch": round(dt * 1e3, 3),
            "mpix_per_s": round(mpix / dt, 2), "graph": True}


def schedule_leg(ff, torch, img1, img2, params, pair, reps=20):
    """Flow Fields+ (Sec. 3.3: 4 steps at R+ = 2R, then 8 at R on every scale),
    Flow Fields+ Fast (Sec. 3.4: only 4 steps at R on the finest scale), Fast
    x2 (no finest scale), the rerank of 8 seed candidates (Eq. 4), the serial
    propagation order, the subpixel form and the original schedule checked
    against two backward fields (Sec. 3.7) on the same pair and launch
    tables: Mpix/s and quality."""
    import dataclasses

    import numpy as np

    from ffgen import epe_stats
    res = {}
    plus = dict(iters=8, plus_iters=4, Rp_num=2 * params.R_num)
    for name, kw, n_reps in (("plus", plus, reps), ("plus_fast", dict(plus, fine_iters=4), reps),
                             # Sec. 3.3: a stage of patch scale 3n/2 before every scale below the coarsest
                             ("plus_subscales", dict(plus, subscales=True), 5),
                             # the paper's Flow Fields+ patch radius (Sec. 4.1: r = 4)
                             ("plus_r4", dict(plus, radius=4), reps),
                             # Sec. 3.4: no finest scale, 4 x R on scale 2, one match per 2x2 region
                             ("plus_fast_x2", dict(plus, fine_iters=4, fast_x2=True), reps),
                             # Eq. 4 with the paper's leaf size l = 8 (Sec. 4.1)
                             ("nn_l8", dict(nn_l=8), 5),
                             # serial propagation order (Sec. 3.1), exact by anti-diagonal wavefronts
                             ("raster", dict(raster=True), 2)):
        prm = dataclasses.replace(params, **kw)
        H, W = img1.shape
        runner = ff.FlowFields(W, H, prm, device=img1.device)
        for _ in range(1 if prm.raster else 3):
            runner(img1, img2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_reps):
            runner(img1, img2)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / n_reps * 1e3
        out = runner.out
        # Fast x2's fields sit on the grid of scale 2: judged at its cells' pixels
        g = 2 if prm.fast_x2 else 1
        q = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt[::g, ::g], pair.occ[::g, ::g],
                      keep=out["keep_fwd"].cpu().numpy())
        res[name] = {"mpix_per_s": round(W * H / ms / 1e3, 2), "ms_per_pair": round(ms, 4),
                     "steps": f"{prm.plus_iters} x R+ then {prm.iters} x R"
                              + (f", finest {prm.fine_iters} x R" if prm.fine_iters else "")
                              + (", finest scale skipped, grid of scale 2" if prm.fast_x2 else "")
                              + (", sub-scales 3n/2" if prm.subscales else "")
                              + (f", patch radius {prm.radius}" if prm.radius != params.radius else ""),
                     "n_evals": [int(v) for v in out["n_evals"].cpu()], "epe_raw": round(q["epe"], 4),
                     "le3px": round(q["le3px"], 4), "kept_density": round(q["kept_density"], 4),
                     "kept_epe": round(q["kept_epe"], 4)}
    # subpixel random search (Sec. 3.1): flows in 1/8 px, bilinear targets (per-step kernels)
    import numpy as _np
    prm = dataclasses.replace(params, subpixel=3)
    H, W = img1.shape
    runner = ff.FlowFields(W, H, prm, device=img1.device)
    runner(img1, img2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        runner(img1, img2)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    out = runner.out
    q = epe_stats(out["flow_fwd"].cpu().numpy().astype(_np.float64) / 8.0, pair.flow_gt, pair.occ,
                  keep=out["keep_fwd"].cpu().numpy())
    res["subpixel"] = {"mpix_per_s": round(W * H / ms / 1e3, 2), "ms_per_pair": round(ms, 4),
                       "flow_unit": "1/8 px", "n_evals": [int(v) for v in out["n_evals"].cpu()],
                       "epe_raw": round(q["epe"], 4), "le3px": round(q["le3px"], 4),
                       "kept_density": round(q["kept_density"], 4), "kept_epe": round(q["kept_epe"], 4)}
    # the original schedule with the check against two backward fields (Sec. 3.7; second field: seed + 1,
    # patch radius 2; Sec. 4.1: r = 3, r2 = 2 for the conference approach)
    run2 = lambda: ff.flow_fields_two_backward(img1, img2, params, radius2=2)  # noqa: E731
    for _ in range(3):
        run2()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = run2()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    q = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt, pair.occ, keep=out["keep_fwd"].cpu().numpy())
    H, W = img1.shape
    res["two_backward"] = {"mpix_per_s": round(W * H / ms / 1e3, 2), "ms_per_pair": round(ms, 4),
                           "second_backward": "seed + 1, patch radius 2", "kept_density": round(q["kept_density"], 4),
                           "kept_epe": round(q["kept_epe"], 4)}
    # then the region filter (Sec. 3.7, s = 50) and the 3 x 3 sparsification (Sec. 3.8, e = 2) on that field
    def filters():
        kf = ff.region_filter(out["flow_fwd"], out["cost_fwd"], out["keep_fwd"], 50)
        return kf, ff.sparsify(out["flow_fwd"], kf, out["flow_bwd"], out["flow_bwd2"], 3, 2)
    for _ in range(3):
        filters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        kf, sel = filters()
    torch.cuda.synchronize()
    fms = (time.perf_counter() - t0) / reps * 1e3
    qf = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt, pair.occ, keep=kf.cpu().numpy())
    idx = sel.cpu().numpy().ravel()
    idx = idx[idx >= 0]
    picked = np.zeros((H, W), np.uint8)
    picked.flat[idx] = 1
    qs = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt, pair.occ, keep=picked)  # non-occluded samples
    res["filtered"] = {"ms_region_filter_and_sparsify": round(fms, 4), "region_s": 50, "sparsify_q_e": [3, 2],
                       "kept_density": round(qf["kept_density"], 4), "kept_epe": round(qf["kept_epe"], 4),
                       "samples": int(len(idx)), "sample_epe": round(qs["kept_epe"], 4)}
    return res


def learned_leg(ff, torch, img1, img2, params, pair, plain_ms, args):
    """DescNet trained on the plain method's consistent matches (16 training
    pairs of the learned workload), judged on held-out pairs of that
    workload against the plain field by the mean ground-truth EPE of the
    whole field and of the matches the consistency check keeps (Sec. 3.7),
    with the per-pair spread; fallback to plain when it is worse on either,
    then
    timed on the 1024x436 pair: descriptor network on every scale image of
    both images + learned-feature fields fwd+bwd + consistency."""
    import numpy as np

    from ffgen import epe_stats, make_pair
    from paper_1703_02563_amd import learned as Lm

    def dev_pair(cfg, k):
        p = make_pair(cfg, k)
        return p, torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()

    batch = []
    for k in range(args.train_pairs):
        _, i1, i2 = dev_pair(5, k)
        o = ff.flow_fields(i1, i2, params)
        batch.append((i1, i2, Lm.TripletSampler(o["flow_fwd"], o["keep_fwd"])))
    net = Lm.DescNet(seed=0)
    rng = np.random.default_rng(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for s in range(args.train_steps):
        losses.append(Lm.train_step(net, batch, rng, samples=args.train_samples, lr=args.train_lr))
        if (s + 1) % 20 == 0:
            log(f"bench: learned training step {s + 1} loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def epe(o, p):
        return epe_stats(o["flow_fwd"].cpu().numpy(), p.flow_gt, p.occ, keep=o["keep_fwd"].cpu().numpy())

    # the judge: raw EPE of the whole field and EPE of the matches the
    # consistency check keeps, per held-out pair, plain beside learned
    keys = ("epe", "kept_epe", "le3px", "kept_density")
    val = {"plain": {k: [] for k in keys}, "learned": {k: [] for k in keys}}
    for k in range(args.val_pairs):
        p, i1, i2 = dev_pair(5, args.train_pairs + k)
        for name, o in (("plain", ff.flow_fields(i1, i2, params)),
                        ("learned", Lm.learned_flow_fields(net, i1, i2, params))):
            q = epe(o, p)
            for key in keys:
                val[name][key].append(round(q[key], 4))
    mean = {name: {key: round(float(np.mean(v)), 4) for key, v in d.items()} for name, d in val.items()}
    d_raw = np.subtract(val["learned"]["epe"], val["plain"]["epe"])
    d_kept = np.subtract(val["learned"]["kept_epe"], val["plain"]["kept_epe"])
    worse_raw = mean["learned"]["epe"] > mean["plain"]["epe"]
    worse_kept = mean["learned"]["kept_epe"] > mean["plain"]["kept_epe"]
    fallback = bool(worse_raw or worse_kept)
    verdict = (f"learned {'worse' if worse_raw else 'better or equal'} on mean raw EPE by "
               f"{abs(float(d_raw.mean())):.3f} px (better on {int((d_raw < 0).sum())}/{len(d_raw)} pairs), "
               f"{'worse' if worse_kept else 'better or equal'} on mean kept EPE by {abs(float(d_kept.mean())):.3f} px "
               f"(better on {int((d_kept < 0).sum())}/{len(d_kept)} pairs): "
               f"{'fall back to plain descriptors' if fallback else 'learned descriptors kept'}")

    run = lambda: Lm.learned_flow_fields(net, img1, img2, params)  # noqa: E731
    for _ in range(2):
        run()
    torch.cuda.synchronize()
    reps = max(3, min(args.steps, 20))
    t0 = time.perf_counter()
    for _ in range(reps):
        out = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    scales = Lm.scale_images(img1, img2, params.levels)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        Lm.learned_features(net, scales)
    e1.record()
    torch.cuda.synchronize()
    net_ms = e0.elapsed_time(e1) / reps
    q = epe(out, pair)
    H, W = img1.shape
    return {"mpix_per_s": round(W * H / ms / 1e3, 2), "ms_per_pair": round(ms, 3),
            "descnet_ms": round(net_ms, 3), "ratio_vs_plain": round(plain_ms / ms, 4),
            "epe_raw": round(q["epe"], 4), "le3px": round(q["le3px"], 4), "kept_epe": round(q["kept_epe"], 4),
            "kept_density": round(q["kept_density"], 4),
            "val_pairs": args.val_pairs, "val_per_pair": val, "val_mean": mean,
            "val_learned_minus_plain": {"epe": [round(float(v), 4) for v in d_raw],
                                        "kept_epe": [round(float(v), 4) for v in d_kept]},
            "verdict": verdict, "fallback_to_plain": fallback,
            "train_pairs": args.train_pairs, "train_steps": args.train_steps,
            "train_samples_per_pair": args.train_samples, "train_s": round(train_s, 2),
            "loss_first_last": [round(losses[0], 5), round(losses[-1], 5)] if losses else None,
            "dtype": "bf16 network, f32 cost"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-pair measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-descriptor measurement")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the Flow Fields+ / Fast / two-backward-field measurements")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 160x120 and 1242x375 pairs (GPU beside the oracle)")
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--val-pairs", type=int, default=8, help="held-out pairs of the EPE judge")
    ap.add_argument("--train-pairs", type=int, default=16)
    ap.add_argument("--train-samples", type=int, default=1024, help="triplets per training pair and step")
    ap.add_argument("--train-lr", type=float, default=1e-3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the Flow Fields pair workload is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1703_02563_amd as ff
    from ffgen import CONFIG_PARAMS, epe_stats, make_pair

    cfg = 2
    pair = make_pair(cfg)
    c = CONFIG_PARAMS[cfg]
    H, W = pair.img1.shape
    params = ff.Params(levels=c.levels, iters=c.iters, radius=c.radius, R_num=c.R_num, R_den=c.R_den, eps=c.eps,
                       seed=c.seed)
    dev = torch.device("cuda:0")
    img1 = torch.from_numpy(pair.img1).to(dev)
    img2 = torch.from_numpy(pair.img2).to(dev)
    import dataclasses

    from paper_1703_02563_amd import autotune
    tuned = autotune.load(W, H, params)
    if tuned is not None:
        params = dataclasses.replace(params, tuning=tuned)
    tun = params.tuning or ff.default_tuning()
    log(f"bench: level-kernel variants {tun.variant}, passes per launch {tun.passes} "
        f"({'tuned' if tuned else 'defaults'}; "
        f"cache {autotune.DEFAULT_CACHE}, key {autotune._key(W, H, params)})")
    runner = ff.FlowFields(W, H, params, device=dev)
    log(f"bench: {W}x{H} L={c.levels} T={c.iters}, warmup {args.warmup}")
    for _ in range(args.warmup):
        runner(img1, img2)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runner(img1, img2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = W * H * args.steps / dt / 1e6
    out = runner.out
    n_evals = [int(v) for v in out["n_evals"].cpu()]
    q = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt, pair.occ, keep=out["keep_fwd"].cpu().numpy())
    log(f"bench: {ms:.3f} ms/step, {value:.1f} Mpix/s, n_evals {n_evals}, quality {q}")

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {nbytes} bytes")

    schedules = None
    if not args.no_schedules:
        log("bench: Flow Fields+ schedules")
        schedules = schedule_leg(ff, torch, img1, img2, params, pair)
        log(f"bench: schedules {schedules}")

    batched = None
    if not args.no_batch:
        log("bench: batched 64-pair workload (graph replay)")
        batched = batched_throughput(ff, torch, reps=5)
        log(f"bench: batched {batched}")

    learned = None
    if not args.no_learned:
        log(f"bench: learned descriptors ({args.train_steps} training steps on {args.train_pairs} pairs)")
        learned = learned_leg(ff, torch, img1, img2, params, pair, ms, args)
        log(f"bench: learned {learned}")

    log("bench: roofline of the scale-1 level kernel")
    roof = roofline_level0(ff, torch, img1, img2, params, reps=20)
    log(f"bench: roofline {roof}")

    threads = max(1, min(16, os.cpu_count() or 1))
    legs = None
    if not args.no_configs:
        log("bench: other single-pair workloads, GPU beside the oracle")
        legs = config_legs(ff, torch, threads)
        log(f"bench: configs {legs}")

    base = None
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline on {threads} threads and on 1 thread")
        base = cpu_baseline(pair, c, threads)

    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "plain Flow Fields, one 1024x436 uint8 pair (12 polygon layers, t in +-150 px), "
                               "16-ch uint8 descriptors, 7x7 SAD, 5 scales x 6 steps, fwd+bwd+consistency",
                   "W": W, "H": H, "levels": c.levels, "iters": c.iters, "R": f"{c.R_num}/{c.R_den}",
                   "n_evals": n_evals, "epe_raw": round(q["epe"], 4), "le3px": round(q["le3px"], 4),
                   "epe10": round(q["epe10"], 4), "kept_density": round(q["kept_density"], 4),
                   "kept_epe": round(q["kept_epe"], 4), "schedules": schedules, "batched": batched,
                   "learned": learned, "other_pairs": legs},
        "roofline": roof,
        "nn_counters": nn_counters(),
        "cpu_baseline": base,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
