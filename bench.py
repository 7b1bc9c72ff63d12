"""Benchmark of the FDTD hot path on one MI355X.

A step is one full forward modelling of the marine layered workload
(128 x 128 x 96 nodes, 162 x 162 x 130 padded cells, 3 frequencies,
101 receivers x 6 channels, one x-dipole): per-forward set-up, every time
step (E step with injection and H-channel DTFT, H step with E-channel DTFT)
and the Green's-function normalisation.  The model is created (and its
arrays uploaded) before the timed region.

Prints one JSON line: Gcell.step/s (padded cells x time steps / wall time),
the roofline of the dominant kernel (E step: algorithmic bytes / average
kernel duration from HIP events recorded around every launch in the timed
region), and the FP64 oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import subprocess
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of one E-step launch on the marine workload, measured with
# rocprofv3 --pmc FETCH_SIZE (x 2.0) and --pmc WRITE_SIZE (x 1.0), the factors
# from a 1 GiB copy kernel: 54 421.1 KiB read and 46 143.4 KiB written (32 x 8
# tiles, 5 planes per block, compact dt/eps).  Valid for the kernel as
# profiled; None when the kernel has changed since, until re-measured.
E_STEP_TRAFFIC_BYTES = (54421.1 * 2.0 + 46143.4 * 1.0) * 1024
# the same for one launch of the fused step kernel (None until measured)
LEAP_TRAFFIC_BYTES = None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, nt_sample: int):
    from oracle import forward as F
    threads = min(16, os.cpu_count() or 1)
    F.forward(w, threads=threads, nt=2)       # load + warm
    t = time.perf_counter()
    F.forward(w, threads=threads, nt=nt_sample)
    dt = time.perf_counter() - t
    cells = w.padded_cells
    return {"value": cells * nt_sample / dt / 1e9, "unit": "Gcell*step/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{w.name}, first {nt_sample} time steps, FP64 C/OpenMP oracle, "
                      f"{dt:.1f} s wall"}


def stream_reference(reps: int = 20):
    """A plain streaming rate measured on this GPU: torch's device copy of a
    1 GiB array (read + write), timed with events after a warm-up."""
    import torch
    a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    sec = t0.elapsed_time(t1) / 1e3 / reps
    nbytes = 2 * a.numel() * 4
    del a, b
    torch.cuda.empty_cache()
    return {"kernel": "device copy of 1 GiB (torch copy_)", "GBs": nbytes / sec / 1e9}


def batched_comparison(emm, w, nsrc: int, group: int, ckpt: int):
    """16 towed x-dipoles (500 m spacing, 50 m above the seabed) on the same
    model: the plain loop of one-source forwards, one batched forward of all
    sources (sources grouped to stay in the Infinity Cache, and all in one
    time loop), and batched forward + gradient (log misfit against data from
    the batched forward scaled by 1.01) in groups of `group` sources that
    keep checkpoints every `ckpt` steps.  Returns timings and the largest
    difference between batched and plain results."""
    import numpy as np
    from workloads import configs
    src = configs.towline_sources(nsrc, 500.0, 950.0)
    comp = np.zeros(nsrc, dtype=np.int32)
    out = {"sources": nsrc, "gradient_group": group, "checkpoint_every": ckpt}
    with emm.Model(w, tile_kz=-1, graph_steps=64) as m:
        m.forward(sources=src[:1], src_comp=comp[:1])           # tune + warm
        t = time.perf_counter()
        plain = [m.forward(sources=src[i:i + 1], src_comp=comp[i:i + 1]) for i in range(nsrc)]
        out["plain_forward_loop_s"] = time.perf_counter() - t
        m.forward(sources=src, src_comp=comp)                   # tune for the group + warm
        t = time.perf_counter()
        Gb = m.forward(sources=src, src_comp=comp)
        out["batched_forward_s"] = time.perf_counter() - t
        out["batched_sources_per_time_loop"] = m.info()["src_group"]
    # all sources in one time loop (every launch updates all of them)
    with emm.Model(w, tile_kz=-1, graph_steps=64, src_group=-1) as m:
        m.forward(sources=src, src_comp=comp)                   # tune for nsrc + warm
        t = time.perf_counter()
        G1 = m.forward(sources=src, src_comp=comp)
        out["one_loop_forward_s"] = time.perf_counter() - t
    Gp = np.concatenate(plain, axis=0)
    out["max_abs_diff_batched_vs_plain"] = float(max(np.max(np.abs(Gb - Gp)), np.max(np.abs(G1 - Gp))))
    G_obs = Gb * 1.01
    with emm.Model(w, tile_kz=-1, checkpoint_every=ckpt, graph_steps=64) as m:
        m.forward(sources=src[:group], src_comp=comp[:group])   # tune + warm
        t = time.perf_counter()
        for g0 in range(0, nsrc, group):
            sl = slice(g0, min(nsrc, g0 + group))
            m.forward(sources=src[sl], src_comp=comp[sl])
            m.gradient(g_obs=G_obs[sl], sources=src[sl], src_comp=comp[sl])
        out["batched_forward_gradient_s"] = time.perf_counter() - t
    out["speedup_batched_forward_vs_plain_loop"] = out["plain_forward_loop_s"] / out["batched_forward_s"]
    out["speedup_one_loop_vs_plain_loop"] = out["plain_forward_loop_s"] / out["one_loop_forward_s"]
    out["batched_fwd_grad_over_plain_forward_loop"] = (out["batched_forward_gradient_s"] /
                                                       out["plain_forward_loop_s"])
    return out


def multi_model_comparison(emm, graph: int):
    """Eight seeded layered + box models from 64^3 to 160 x 160 x 120 nodes
    (each with its own dt and step count): their forwards one after another
    versus emm_forward_batch (jobs grouped into graphs by the cache budget)
    and versus all of them as branches of one hipGraph."""
    import numpy as np
    from workloads import configs
    ws = configs.batched_models()
    models = [emm.Model(w, tile_kz=-1, graph_steps=graph) for w in ws]
    # the same first model with src_group = -1: as the first job it puts
    # every job into one group (all side by side)
    first_all = emm.Model(ws[0], tile_kz=-1, graph_steps=graph, src_group=-1)
    try:
        for m in models + [first_all]:                         # tune + warm
            m.forward()
        t = time.perf_counter()
        seq = [m.forward() for m in models]
        t_seq = time.perf_counter() - t
        emm.forward_models(models, graph_steps=graph)          # warm
        t = time.perf_counter()
        bat = emm.forward_models(models, graph_steps=graph)
        t_bat = time.perf_counter() - t
        groups = [m.info()["src_group"] for m in models]
        emm.forward_models([first_all] + models[1:], graph_steps=graph)   # warm
        t = time.perf_counter()
        one = emm.forward_models([first_all] + models[1:], graph_steps=graph)
        t_one = time.perf_counter() - t
        cellsteps = sum(m.info()["cells"] * m.info()["nt"] for m in models)
    finally:
        for m in models + [first_all]:
            m.close()
    same = all(np.array_equal(a, b) and np.array_equal(a, c) for a, b, c in zip(seq, bat, one))
    # eight small grids (74^3 padded), which one at a time leave most of the chip idle
    small = [configs.uniform_cube(40, nt=640) for _ in range(8)]
    sm = [emm.Model(w, graph_steps=graph) for w in small]
    try:
        for m in sm:
            m.forward()
        t = time.perf_counter()
        for m in sm:
            m.forward()
        s_seq = time.perf_counter() - t
        emm.forward_models(sm, graph_steps=graph)
        t = time.perf_counter()
        emm.forward_models(sm, graph_steps=graph)
        s_bat = time.perf_counter() - t
        s_grp = sm[0].info()["src_group"]
    finally:
        for m in sm:
            m.close()
    return {"small_models": {"models": "8 x uniform_cube_40 (74^3 padded), 640 steps",
                             "sequential_s": s_seq, "batch_s": s_bat, "speedup": s_seq / s_bat,
                             "jobs_per_graph": s_grp},
            "models": [w.name for w in ws], "sequential_s": t_seq, "batch_s": t_bat,
            "jobs_per_graph": groups, "speedup": t_seq / t_bat, "all_in_one_graph_s": t_one,
            "speedup_all_in_one_graph": t_seq / t_one, "gcell_steps": cellsteps / 1e9,
            "batch_gcell_step_per_s": cellsteps / t_bat / 1e9, "bitwise_equal": same}


def large_fwd_grad(emm, nt: int, group: int, graph: int):
    """The 400 x 400 x 200 marine grid at 8th order (438 x 438 x 238 padded
    cells), 8 x-dipoles, 400 receivers, 5 frequencies, compensated FP32 DTFT:
    plain loop of one-source forwards, one batched forward of the 8
    sources, and forward + gradient (log misfit against the batched result
    scaled by 1.01) in groups of `group` sources, each under the planned
    checkpoint schedule."""
    from workloads import configs
    w = configs.large_marine(nt=nt, rd=4, nsrc=8)
    out = {"workload": w.name, "time_steps": nt, "sources": 8, "gradient_group": group}
    with emm.Model(w, tile_kz=-1, graph_steps=graph) as m:
        m.forward(sources=w.sources[:1], src_comp=w.src_comp[:1])         # tune + warm
        t = time.perf_counter()
        for s in range(8):
            m.forward(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1])
            log(f"[bench] large: plain forward of source {s} done")
        out["plain_forward_loop_s"] = time.perf_counter() - t
        m.forward()                                                     # tune for 8 + warm
        log("[bench] large: batched warm-up done")
        t = time.perf_counter()
        Gb = m.forward()
        out["batched_forward_s"] = time.perf_counter() - t
        log("[bench] large: batched forward done")
        G_obs = Gb * 1.01
        sched = []
        t = time.perf_counter()
        for g0 in range(0, 8, group):
            sl = slice(g0, min(8, g0 + group))
            m.gradient(g_obs=G_obs[sl], sources=w.sources[sl], src_comp=w.src_comp[sl])
            i = m.info()
            sched.append([i["ckpt_outer"], i["ckpt_inner"], i["ckpt_bytes"] / 2 ** 30, i["src_group"]])
            log(f"[bench] large: gradient of sources {g0}..{sl.stop - 1} done, schedule {sched[-1]}")
        out["forward_gradient_s"] = time.perf_counter() - t
        out["checkpoint_schedule_outer_inner_GiB_sources_per_sweep"] = sched
        out["cells"] = m.info()["cells"]
    out["batched_forward_vs_plain_loop"] = out["plain_forward_loop_s"] / out["batched_forward_s"]
    out["forward_gradient_over_plain_forward_loop"] = out["forward_gradient_s"] / out["plain_forward_loop_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2000)
    ap.add_argument("--workload", default="marine", choices=["marine", "large", "cube", "shallow"],
                    help="marine: the headline 128x128x96 workload; large: the 400x400x200 "
                         "marine grid (one source); cube: uniform n^3 (--cube-n); shallow: "
                         "128x128x80 shallow water with the air boundary")
    ap.add_argument("--cube-n", type=int, default=400)
    ap.add_argument("--rd", type=int, default=0, help="override the stencil half length")
    ap.add_argument("--nt", type=int, default=0, help="override the time-step count")
    ap.add_argument("--graph", type=int, default=64, help="time steps per captured hipGraph (0: direct launches)")
    ap.add_argument("--fused", type=int, default=0, choices=[0, 1],
                    help="1: one fused launch per time step (E and H updates)")
    ap.add_argument("--tile-kz", type=int, default=-1, help="z planes per block (-1: autotuned)")
    ap.add_argument("--tile-x", type=int, default=0, choices=(0, 32, 64),
                    help="columns per block of the stencil kernels (0: autotuned or by the grid)")
    ap.add_argument("--batched", type=int, default=16,
                    help="sources of the batched comparison (0: skip)")
    ap.add_argument("--grad-group", type=int, default=8)
    ap.add_argument("--grad-ckpt", type=int, default=128)
    ap.add_argument("--no-multi-model", action="store_true",
                    help="skip timing 8 models of uneven sizes in one hipGraph vs one after another")
    ap.add_argument("--large-fwd-grad", type=int, default=0, metavar="NT",
                    help="also time the 8-source 8th-order forward + gradient on the 400x400x200 "
                         "grid with NT time steps (0: skip)")
    ap.add_argument("--large-group", type=int, default=8,
                    help="sources per emm_gradient call of --large-fwd-grad (the library then "
                         "groups them per sweep by its checkpoint plan)")
    ap.add_argument("--gradient-sample", type=int, default=0, metavar="NT",
                    help="only run one forward + gradient of the marine (or, with --workload "
                         "large, the large-grid) workload cut to NT steps (for kernel traces of "
                         "the adjoint) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy kernel (for scaling FETCH/WRITE_SIZE)")
    ap.add_argument("--stream-reference", action="store_true",
                    help="print the device-copy rate of this GPU as JSON and exit")
    args = ap.parse_args()
    if args.stream_reference:
        print(json.dumps(stream_reference()))
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {a.numel() * 4} bytes")
        return
    if args.gradient_sample:
        from paper_2304_00233_amd import emm
        from workloads import configs
        if args.workload == "large":
            w = configs.large_marine(nt=args.gradient_sample, rd=args.rd or 4, nsrc=1)
        else:
            w = configs.marine_layered(nt=args.gradient_sample)
        with emm.Model(w, tile_kz=-1, graph_steps=64) as m:
            G = m.forward()
            t = time.perf_counter()
            m.gradient(g_obs=G * 1.01)
            dt = time.perf_counter() - t
            i = m.info()
        log(f"[bench] gradient sample: {w.name}, {args.gradient_sample} steps, forward + gradient "
            f"{dt * 1e3:.1f} ms, checkpoints every {i['ckpt_outer']} (inner {i['ckpt_inner']})")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path shards by "
              "source with no communication between GPUs", file=sys.stderr)
        sys.exit(2)

    # the streaming reference runs in a child process before this one touches
    # the GPU (torch brings its own HIP runtime, which cannot share a process
    # with the library's)
    stream_ref = None
    try:
        log("[bench] stream reference (1 GiB device copy, child process)")
        res = subprocess.run([sys.executable, os.path.abspath(__file__), "--stream-reference"],
                             capture_output=True, text=True, timeout=300)
        if res.returncode == 0:
            stream_ref = json.loads(res.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        stream_ref = None

    from paper_2304_00233_amd import emm
    from workloads import configs

    if args.workload == "marine":
        w = configs.marine_layered()
        nt = 0
        gold = os.path.join(ROOT, "tests", "golden", "marine_layered_oracle.json")
        if os.path.exists(gold):
            nt = json.load(open(gold))["nt"]
        w = w.with_(nt=nt)
    elif args.workload == "shallow":
        w = configs.shallow_marine()
        gold = os.path.join(ROOT, "tests", "golden", "shallow_marine_air_oracle.json")
        if os.path.exists(gold):
            w = w.with_(nt=json.load(open(gold))["nt"])
    elif args.workload == "large":
        w = configs.large_marine(nsrc=1).with_(dft_mode=0)
    else:
        w = configs.uniform_cube(args.cube_n)
    if args.rd:
        w = w.with_(rd=args.rd, ne=args.rd + 5)
    if args.nt:
        w = w.with_(nt=args.nt)
    log(f"[bench] workload {w.name} padded cells {w.padded_cells}")

    model = emm.Model(w, profile=1, graph_steps=args.graph, tile_kz=args.tile_kz, fused=args.fused,
                      tile_x=args.tile_x)
    for i in range(args.warmup):
        model.forward()
        log(f"[bench] warmup {i} done")
    e_ms = h_ms = 0.0
    e_n = h_n = 0
    dev_ms = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        model.forward()
        inf = model.info()
        e_ms += inf["e_kernel_ms"]
        h_ms += inf["h_kernel_ms"]
        e_n += inf["e_launches"]
        h_n += inf["h_launches"]
        dev_ms += inf["forward_ms"]
    wall = time.perf_counter() - t0
    info = model.info()
    model.close()
    nt = info["nt"]
    cells = info["cells"]
    ms_per_step = wall / args.steps * 1e3
    value = cells * nt * args.steps / wall / 1e9
    e_avg_s = e_ms / e_n / 1e3 if e_n else float("nan")
    h_avg_s = h_ms / h_n / 1e3 if h_n else float("nan")
    fused = bool(info["fused"])
    kbytes = info["leap_bytes"] if fused else info["e_bytes"]
    achieved = kbytes / e_avg_s / 1e9
    log(f"[bench] nt={nt} wall/forward={ms_per_step:.1f} ms device loop/forward="
        f"{dev_ms / args.steps:.1f} ms e_step avg={e_avg_s * 1e6:.2f} us "
        f"h_step avg={h_avg_s * 1e6:.2f} us tile_kz={info['tile_kz']} tile_x={info['tile_x']} "
        f"nontemporal={info['nontemporal']} ce_table={info['ce_table']}")
    out = {
        "metric": "FDTD cell-updates/s (Gcell*step/s) + % HBM peak",
        "value": value, "unit": "Gcell*step/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (fields), f64 (DFT)",
        "data": "synthetic",
        "config": {"workload": w.name, "padded_cells": cells, "time_steps": nt,
                   "rd": w.rd, "sources": len(w.sources), "receivers": len(w.receivers),
                   "channels": 6, "freqs": [float(f) for f in w.freqs],
                   "step": "one full forward modelling (nt time steps)"},
        "roofline": {"bound": "hbm",
                     "kernel": ("leap (E update + H update of one step, E on the halo recomputed, "
                                "J, CPML, DTFT)") if fused else
                               "e_step (curl H + CPML + J + E update + H DTFT)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (LEAP_TRAFFIC_BYTES if fused else E_STEP_TRAFFIC_BYTES)
                     if args.workload == "marine" else None,
                     "bytes_per_launch": kbytes, "avg_launch_us": e_avg_s * 1e6},
        "device_loop_ms_per_step": dev_ms / args.steps,
        # the same run counted over the model's interior nodes only (the
        # padding of nb + ne cells per face is streamed too, so `value`
        # counts it)
        "interior_gcell_step_per_s": (len(w.x1) * len(w.x2) * len(w.x3)) * nt * args.steps / wall / 1e9,
        "launch": {"tile_kz": info["tile_kz"], "tile_x": info["tile_x"],
                   "nontemporal": info["nontemporal"], "compact_dt_eps": info["ce_table"],
                   "graph_steps": args.graph},
        "fused_step": fused,
    }
    if not fused:
        out["h_step"] = {"bytes_per_launch": info["h_bytes"], "avg_launch_us": h_avg_s * 1e6,
                         "achieved_GBs": info["h_bytes"] / h_avg_s / 1e9}
    if stream_ref:
        out["stream_reference"] = dict(stream_ref)
        out["stream_reference"]["e_step_frac_of_it"] = achieved / stream_ref["GBs"]
    if args.batched and args.workload == "marine":
        log(f"[bench] batched comparison with {args.batched} sources")
        out["batched"] = batched_comparison(emm, w, args.batched, args.grad_group, args.grad_ckpt)
        log(f"[bench] batched: {out['batched']}")
    if not args.no_multi_model and args.workload == "marine":
        log("[bench] multi-model comparison")
        out["multi_model"] = multi_model_comparison(emm, args.graph or 64)
        log(f"[bench] multi-model: {out['multi_model']}")
    if args.large_fwd_grad:
        log(f"[bench] large 8-source forward + gradient, {args.large_fwd_grad} steps")
        out["large_fwd_grad"] = large_fwd_grad(emm, args.large_fwd_grad, args.large_group,
                                               args.graph or 64)
        log(f"[bench] large: {out['large_fwd_grad']}")
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
