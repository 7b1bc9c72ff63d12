"""Benchmark of the FDTD hot path on one MI355X.

Default workload: the large marine grid (400 x 400 x 200 nodes, 438 x 438 x
238 padded cells), 8th order in space, 8 towed x-dipoles in one batched
launch per half step, 400 seafloor receivers x 6 channels, 5 frequencies
0.1..2 Hz, FP32 fields with the compensated FP32 DTFT.  A step is one
emm_forward of the 8 sources over a window of --window time steps (every
row of the hot path: per-forward set-up, E step with injection and H-channel
DTFT, H step with E-channel DTFT, Green's-function normalisation); the
model is created (and its arrays uploaded) before the timed region.

Prints one JSON line: source-cell updates per second (padded cells x time
steps x sources / wall time), the roofline of the dominant kernel (the E
step: algorithmic bytes per launch / its average duration from HIP events
that the dispatch stamps at kernel start and end, sampled in the timed
region), the batched forward + gradient against the plain one-source loops,
the accuracy of the FP32 path against the stored FP64 oracle result of one
source at the full step count, and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LARGE_GOLDEN = os.path.join(ROOT, "tests", "golden", "large_marine_oracle.json")
MARINE_GOLDEN = os.path.join(ROOT, "tests", "golden", "marine_layered_oracle.json")
SHALLOW_GOLDEN = os.path.join(ROOT, "tests", "golden", "shallow_marine_air_oracle.json")
PLAIN_GOLDEN = os.path.join(ROOT, "tests", "golden", "plain_forward_48cube_oracle.json")

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE (x 2.0) and WRITE_SIZE
# (x 1.0), the factors from a 1 GiB copy kernel, keyed by workload, kernel and
# launch configuration (tile width, rows per wavefront, source order,
# nontemporal hint, compact dt/eps, sources, z planes per block).  A run whose
# autotuned launch differs reports null: the counters belong to the kernel as
# profiled.
TRAFFIC_KIB = {
    # (workload, kernel, tx, ry, source order, nontemporal, compact, nsrc, kz):
    #     (FETCH_SIZE KiB, WRITE_SIZE KiB); the large grid at 8th order with 8
    #     sources (profiles/step_kernel_large_marine_*)
    ("large_marine_400x400x200", "e_step", 32, 1, 1, 0, 1, 8, 58): (6401647.6, 4453677.2),
    ("large_marine_400x400x200", "h_step", 32, 1, 1, 0, 1, 8, 58): (5792745.6, 4453299.9),
    ("large_marine_400x400x200", "e_step", 64, 1, 1, 0, 1, 8, 58): (6574432.7, 4450545.0),
    ("large_marine_400x400x200", "h_step", 64, 1, 1, 0, 1, 8, 58): (5874936.8, 4454413.7),
    ("large_marine_400x400x200", "e_step", 32, 1, 1, 1, 1, 8, 58): (5845896.3, 4449371.8),
    ("large_marine_400x400x200", "h_step", 32, 1, 1, 1, 1, 8, 58): (5187237.2, 4451036.2),
    ("large_marine_400x400x200", "e_step", 64, 1, 1, 1, 1, 8, 58): (5762863.4, 4433150.8),
    ("large_marine_400x400x200", "h_step", 64, 1, 1, 1, 1, 8, 58): (5067565.9, 4436068.8),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cores():
    """Cores this process may use: its CPU affinity, capped by a cgroup CPU
    quota when one is set; plus the CPU model name."""
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, int(-(-int(q) // int(per))))
    except (OSError, ValueError):
        pass
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": aff, "cgroup_quota_cpus": quota,
            "usable": min(aff, quota) if quota else aff, "model": model}


def cpu_baseline(w, steps_all: int, steps_one: int):
    """The FP64 oracle (C/OpenMP, one source) on the host: all usable cores
    over `steps_all` time steps and one thread over `steps_one`."""
    from oracle import forward as F
    hc = host_cores()
    w1 = w.with_(sources=w.sources[:1], src_comp=w.src_comp[:1])
    cells = w1.padded_cells
    out = {"unit": "Gcell*step/s", "kind": "oracle", "cpu": hc}

    def rate(threads, steps):
        F.forward(w1, threads=threads, nt=1)          # load, set-up and first touch
        t = time.perf_counter()
        F.forward(w1, threads=threads, nt=steps)
        dt = time.perf_counter() - t
        t = time.perf_counter()
        F.forward(w1, threads=threads, nt=1)          # the per-call set-up alone
        setup = time.perf_counter() - t
        return cells * (steps - 1) / max(1e-9, dt - setup) / 1e9, dt
    log(f"[bench] oracle on {hc['usable']} cores, {steps_all} steps")
    v_all, t_all = rate(hc["usable"], steps_all)
    log(f"[bench] oracle on 1 core, {steps_one} steps")
    v_one, t_one = rate(1, steps_one)
    out.update({"value": v_all, "cores": hc["usable"], "one_thread_value": v_one,
                "sample": f"{w.name}, one source, FP64 C/OpenMP oracle: {steps_all} time steps on "
                          f"{hc['usable']} threads ({t_all:.1f} s wall) and {steps_one} steps on 1 "
                          f"thread ({t_one:.1f} s); rate over the steps after the first, the "
                          f"per-call set-up subtracted"})
    return out


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


def kernel_bytes(info, nsrc):
    """Bytes of one E-step and one H-step launch over nsrc sources:
    the section-8(d) count (FP32 dt/eps read once: (36 S + 12) N for the E
    step, 36 S N for the H step, + 16 B per CPML slab cell per axis per
    source) and the bytes the launch moves (the E step reads 4 B of compact
    dt/eps per cell instead of 12 when it uses that form)."""
    N = float(info["cells"])
    e1 = float(info["e_bytes"])          # one source, as the run moved them
    ce_one = (4.0 if info["ce_table"] else 12.0) * N
    per_src_e = e1 - ce_one
    per_src_h = float(info["h_bytes"])
    return {"e_8d": nsrc * per_src_e + 12.0 * N, "e_moved": nsrc * per_src_e + ce_one,
            "h": nsrc * per_src_h}


def traffic(workload, kernel, info, nsrc):
    key = (workload, kernel, info["tile_x"], info["tile_rows"], info["src_order"],
           info["nontemporal"], info["ce_table"], nsrc, info["tile_kz"])
    kib = TRAFFIC_KIB.get(key)
    if kib is None:
        return None
    return (kib[0] * FETCH_SCALE + kib[1] * WRITE_SCALE) * 1024.0


def timed_forwards(m, steps, warmup, label):
    for i in range(warmup):
        m.forward()
        log(f"[bench] {label} warmup {i} done")
    acc = dict(e_ms=0.0, h_ms=0.0, e_n=0, h_n=0, dev_ms=0.0, walls=[])
    t0 = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        m.forward()
        acc["walls"].append(time.perf_counter() - t1)
        inf = m.info()
        acc["e_ms"] += inf["e_kernel_ms"]
        acc["h_ms"] += inf["h_kernel_ms"]
        acc["e_n"] += inf["e_launches"]
        acc["h_n"] += inf["h_launches"]
        acc["dev_ms"] += inf["forward_ms"]
    wall = time.perf_counter() - t0
    log(f"[bench] {label}: {steps} timed steps in {wall:.2f} s")
    return wall, acc, m.info()


def accuracy_vs_golden(emm, gold_path, wl, label, **opt):
    """One source of the workload at the stored result's full step count,
    FP64 and compensated-FP32 accumulators, against the FP64 oracle result:
    per-result amplitude and phase error above the noise floor (max, p99,
    count below the floor)."""
    import numpy as np
    from tests.parity import compare
    g = json.load(open(gold_path))
    G_o = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    s = g.get("source_index", 0)
    w1 = wl.with_(sources=wl.sources[s:s + 1], src_comp=wl.src_comp[s:s + 1], nt=g["nt"])
    out = {"oracle": os.path.relpath(gold_path, ROOT), "time_steps": g["nt"], "source_index": s}
    for mode, name in ((1, "fp32_kahan"), (0, "fp64")):
        t = time.perf_counter()
        with emm.Model(w1.with_(dft_mode=mode), tile_kz=-1, graph_steps=64, **opt) as m:
            G = m.forward()
        rep = compare(G, G_o, g["channels"])
        rep["forward_s"] = time.perf_counter() - t
        out[name] = rep
        log(f"[bench] {label} accuracy {name}: {rep}")
    return out


def plain_accuracy(emm):
    """The plain-forward 48^3 model (1 ohm-m whole space, x-dipole at the
    origin, 21 inline and 6 off-axis receivers, 1 Hz) at the stored result's
    step count with FP64 and compensated-FP32 accumulators: every channel
    against the stored FP64 oracle result, and every field component against
    the analytic whole-space dipole at the receivers 400 m or more from the
    source, where it is at least 1 % of the largest component of its field at
    that receiver (the scheme's discretisation error on 100 m cells, not a
    parity figure)."""
    import numpy as np
    from tests.parity import compare
    from workloads import configs
    g = json.load(open(PLAIN_GOLDEN))
    G_o = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    nrec = g["shape"][1]
    an = (np.array(g["analytic_re"], dtype=float) + 1j * np.array(g["analytic_im"], dtype=float))
    an = an.reshape(nrec, 6)
    far = np.array(g["receiver_distance_m"]) >= 400.0
    use = np.zeros((nrec, 6), dtype=bool)
    for f in (slice(0, 3), slice(3, 6)):
        mag = np.abs(np.nan_to_num(an[:, f]))          # none on the source
        use[:, f] = far[:, None] & (mag > 0.0) & (mag >= 1e-2 * mag.max(axis=1, keepdims=True))
    w = configs.plain_forward_offaxis(nt=g["nt"])
    out = {"oracle": os.path.relpath(PLAIN_GOLDEN, ROOT), "time_steps": g["nt"],
           "analytic_results": int(use.sum())}
    for mode, name in ((1, "fp32_kahan"), (0, "fp64")):
        with emm.Model(w.with_(dft_mode=mode), graph_steps=64) as m:
            G = m.forward()
            dt = m.info()["dt"]
        rep = compare(G, G_o, g["channels"])
        ratio = G[0, :, :, 0][use] / an[use]
        amp, ph = np.abs(np.abs(ratio) - 1.0), np.abs(np.degrees(np.angle(ratio)))
        rep["dt_equal"] = bool(dt == g["dt"])
        rep["analytic_amp_max"] = float(amp.max())
        rep["analytic_amp_median"] = float(np.median(amp))
        rep["analytic_phase_max_deg"] = float(ph.max())
        out[name] = rep
        log(f"[bench] 48^3 accuracy {name}: {rep}")
    return out


def large_batched(emm, w, window, t_batched_fwd):
    """8 sources on the large grid over `window` steps: the plain loop of
    one-source forwards, the batched forward (the benchmark step), the
    batched forward + gradient (of L = 1/2 sum |G|^2, given by its cotangent
    G: within a window shorter than a converged run the far receivers still
    read exactly zero, where a log misfit is undefined; sources grouped per
    sweep by the library's checkpoint plan), and the one-source-at-a-time
    forward + gradient loop."""
    import numpy as np
    nsrc = len(w.sources)
    out = {"sources": nsrc, "time_steps": window, "batched_forward_s": t_batched_fwd}
    with emm.Model(w, tile_kz=-1, graph_steps=64, profile=1) as m:
        m.forward(sources=w.sources[:1], src_comp=w.src_comp[:1])        # tune for 1 + warm
        t = time.perf_counter()
        plain, k = [], dict(e_ms=0.0, h_ms=0.0, e_n=0, h_n=0)
        for s in range(nsrc):
            plain.append(m.forward(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1]))
            i1 = m.info()
            for a, b in (("e_ms", "e_kernel_ms"), ("h_ms", "h_kernel_ms"), ("e_n", "e_launches"),
                         ("h_n", "h_launches")):
                k[a] += i1[b]
        out["plain_forward_loop_s"] = time.perf_counter() - t
        log(f"[bench] large: plain forward loop {out['plain_forward_loop_s']:.2f} s")
        # the one-source kernels of that loop against the peak (section-8(d)
        # bytes of one source: its dt/eps counted in full)
        kb1 = kernel_bytes(i1, 1)
        one = {"launch": {q: i1[q] for q in ("tile_kz", "tile_x", "tile_rows", "src_order",
                                              "nontemporal", "ce_table")}}
        for name, nb, ms, n in (("e_step", kb1["e_8d"], k["e_ms"], k["e_n"]),
                                ("h_step", kb1["h"], k["h_ms"], k["h_n"])):
            us = ms / max(n, 1) * 1e3
            one[name] = {"bytes_per_launch": nb, "avg_launch_us": us, "launches_timed": n,
                         "achieved_GBs": nb / us / 1e3, "frac": nb / us / 1e3 / HBM_PEAK_GBS}
        out["one_source_kernels"] = one
        log(f"[bench] large: one-source E/H {one['e_step']['avg_launch_us']:.1f}/"
            f"{one['h_step']['avg_launch_us']:.1f} us (frac {one['e_step']['frac']:.3f}/"
            f"{one['h_step']['frac']:.3f}), {one['launch']}")
        Gb = m.forward()
        out["batched_equals_plain_bitwise"] = bool(np.array_equal(Gb, np.concatenate(plain, 0)))
        # warm (buffers of the one-source plan) on the last source, so that the
        # first timed call, on another acquisition, runs its own forward
        m.gradient(g_bar=Gb[-1:], sources=w.sources[-1:], src_comp=w.src_comp[-1:])
        t = time.perf_counter()
        for s in range(nsrc):
            m.gradient(g_bar=Gb[s:s + 1], sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1])
        out["plain_forward_gradient_loop_s"] = time.perf_counter() - t
        log(f"[bench] large: one-source forward + gradient loop {out['plain_forward_gradient_loop_s']:.2f} s")
        # the first batched call grows the checkpoint and snapshot buffers to
        # the 8-source plan (~200 GiB of device memory); time the next one,
        # after a plain forward: emm_gradient reuses the checkpoints that the
        # last call left for the same acquisition, and the timed call must
        # run its own forward
        t = time.perf_counter()
        m.gradient(g_bar=Gb)
        out["batched_forward_gradient_first_call_s"] = time.perf_counter() - t
        m.forward()
        t = time.perf_counter()
        m.gradient(g_bar=Gb)
        out["batched_forward_gradient_s"] = time.perf_counter() - t
        t = time.perf_counter()
        m.gradient(g_bar=Gb)
        out["batched_gradient_reusing_checkpoints_s"] = time.perf_counter() - t
        i = m.info()
        out["gradient_sources_per_sweep"] = i["src_group"]
        out["checkpoint_outer_inner"] = [i["ckpt_outer"], i["ckpt_inner"]]
        out["checkpoint_GiB"] = i["ckpt_bytes"] / 2 ** 30
        log(f"[bench] large: batched forward + gradient {out['batched_forward_gradient_s']:.2f} s")
    out["batched_forward_speedup_vs_plain_forward_loop"] = out["plain_forward_loop_s"] / t_batched_fwd
    out["batched_fwd_grad_over_plain_forward_loop"] = (out["batched_forward_gradient_s"] /
                                                       out["plain_forward_loop_s"])
    out["batched_fwd_grad_speedup_vs_plain_fwd_grad_loop"] = (out["plain_forward_gradient_loop_s"] /
                                                             out["batched_forward_gradient_s"])
    return out


def small_towline(emm, nsrc: int = 16):
    """16 x-dipoles every 250 m along x on the 48^3 plain-forward model, all
    in one batched launch per half step, against the plain loop of
    one-source forwards (a launch-bound grid: 82^3 padded cells); then the
    same for forward + gradient (emm_gradient of L = 1/2 sum |G|^2, given by
    its cotangent G, checkpoints every 50 steps): all sources in one sweep
    against one source at a time, with the gradients compared."""
    import numpy as np
    from workloads import configs
    w = configs.towline_small(nsrc)
    out = {"workload": w.name, "sources": nsrc}
    with emm.Model(w, tile_kz=-1, graph_steps=64, src_group=-1) as m:
        m.forward(sources=w.sources[:1], src_comp=w.src_comp[:1])
        m.forward()
        t = time.perf_counter()
        plain = [m.forward(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1]) for s in range(nsrc)]
        out["plain_forward_loop_s"] = time.perf_counter() - t
        t = time.perf_counter()
        Gb = m.forward()
        out["batched_forward_s"] = time.perf_counter() - t
        out["time_steps"] = m.info()["nt"]
    out["bitwise_equal"] = bool(np.array_equal(Gb, np.concatenate(plain, 0)))
    out["speedup"] = out["plain_forward_loop_s"] / out["batched_forward_s"]
    with emm.Model(w, tile_kz=-1, graph_steps=64, src_group=-1, checkpoint_every=50) as m:
        m.gradient(g_bar=Gb[:1], sources=w.sources[:1], src_comp=w.src_comp[:1])    # warm
        m.gradient(g_bar=Gb)
        t = time.perf_counter()
        g_sum = None
        for s in range(nsrc):
            g, _, _ = m.gradient(g_bar=Gb[s:s + 1], sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1])
            g_sum = g if g_sum is None else g_sum + g
        out["plain_forward_gradient_loop_s"] = time.perf_counter() - t
        t = time.perf_counter()
        gb, _, _ = m.gradient(g_bar=Gb)
        out["batched_forward_gradient_s"] = time.perf_counter() - t
        out["gradient_sources_per_sweep"] = m.info()["src_group"]
    out["gradient_max_rel_diff"] = float(np.max(np.abs(gb - g_sum)) / np.max(np.abs(gb)))
    out["fwd_grad_speedup"] = out["plain_forward_gradient_loop_s"] / out["batched_forward_gradient_s"]
    out["batched_fwd_grad_over_plain_forward_loop"] = (out["batched_forward_gradient_s"] /
                                                       out["plain_forward_loop_s"])
    return out


def marine_leg(emm, steps: int):
    """The 128 x 128 x 96 marine layered workload (162 x 162 x 130 padded
    cells, one source, full step count): its working set (~150 MB) sits in
    the 256 MB Infinity Cache, so its bandwidth is an effective (cache-fed)
    figure, not an HBM one."""
    from workloads import configs
    nt = json.load(open(MARINE_GOLDEN))["nt"] if os.path.exists(MARINE_GOLDEN) else 0
    w = configs.marine_layered(nt=nt)
    with emm.Model(w, profile=1, graph_steps=64, tile_kz=-1) as m:
        wall, acc, info = timed_forwards(m, steps, 1, "marine")
    e_us = acc["e_ms"] / max(1, acc["e_n"]) * 1e3
    return {"workload": w.name, "cache_resident": True, "time_steps": info["nt"],
            "gcell_step_per_s": info["cells"] * info["nt"] * steps / wall / 1e9,
            "ms_per_forward": wall / steps * 1e3, "e_step_us": e_us,
            "e_step_effective_GBs": info["e_bytes"] / e_us / 1e3,
            "launch": {"tile_kz": info["tile_kz"], "tile_x": info["tile_x"],
                       "tile_rows": info["tile_rows"], "nontemporal": info["nontemporal"],
                       "compact_dt_eps": info["ce_table"]}}


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



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["large", "marine", "cube", "shallow"],
                    help="large: the 400x400x200 grid at 8th order with 8 batched sources (the "
                         "headline); marine: 128x128x96, one source, full step count; cube: "
                         "uniform n^3 (--cube-n); shallow: 128x128x80 with the air boundary")
    ap.add_argument("--window", type=int, default=256,
                    help="time steps per forward (one benchmark step) of the large workload")
    ap.add_argument("--sources", type=int, default=8, help="sources of the large workload")
    ap.add_argument("--cube-n", type=int, default=400)
    ap.add_argument("--rd", type=int, default=0, help="override the stencil half length")
    ap.add_argument("--nt", type=int, default=0, help="override the time-step count (not large)")
    ap.add_argument("--graph", type=int, default=64, help="time steps per captured hipGraph (0: direct launches)")
    ap.add_argument("--fused", type=int, default=0, choices=[0, 1])
    ap.add_argument("--tile-kz", type=int, default=-1, help="z planes per block (-1: autotuned)")
    ap.add_argument("--tile-x", type=int, default=0, choices=(0, 32, 64))
    ap.add_argument("--tile-rows", type=int, default=0, choices=(0, 1, 2, 4))
    ap.add_argument("--nontemporal", type=int, default=-1, choices=(-1, 0, 1),
                    help="nontemporal hints on the arrays a launch touches once (-1: autotuned)")
    ap.add_argument("--src-order", type=int, default=-1, choices=(-1, 0, 1),
                    help="tile order of the sources (-1: autotuned)")
    ap.add_argument("--air-transform", type=int, default=1, choices=(1, 2, 3),
                    help="air-boundary ghost-fill transforms (shallow workload): 1 by plane size, "
                         "2 hipFFT, 3 direct kernels")
    ap.add_argument("--quick", action="store_true",
                    help="only the timed steps (no batched, accuracy, marine, towline legs)")
    ap.add_argument("--multi-model", action="store_true",
                    help="also time 8 models of uneven sizes side by side (emm_forward_batch) "
                         "against one after another")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=50, help="oracle steps on all cores")
    ap.add_argument("--cpu-steps-one", type=int, default=6, help="oracle steps on one core")
    ap.add_argument("--gradient-sample", type=int, default=0, metavar="NT",
                    help="only run one forward and two gradients (cotangent G; the second timed) of "
                         "the workload cut to NT steps, for kernel traces of the adjoint, and exit")
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
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs on one "
              "device; the path would shard by source with no communication between GPUs",
              file=sys.stderr)
        sys.exit(2)

    # the streaming reference runs in a child process before this one touches
    # the GPU (torch loads its own HIP runtime)
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

    large = args.workload == "large"
    if large:
        rd = args.rd or 4
        w = configs.large_marine(nt=args.window, rd=rd, nsrc=args.sources)
        if rd != 4:
            w = w.with_(ne=rd + 5)
    elif args.workload == "marine":
        nt = json.load(open(MARINE_GOLDEN))["nt"] if os.path.exists(MARINE_GOLDEN) else 0
        w = configs.marine_layered(nt=nt)
    elif args.workload == "shallow":
        w = configs.shallow_marine()
        if os.path.exists(SHALLOW_GOLDEN):
            w = w.with_(nt=json.load(open(SHALLOW_GOLDEN))["nt"])
    else:
        w = configs.uniform_cube(args.cube_n)
    if args.rd and not large:
        w = w.with_(rd=args.rd, ne=args.rd + 5)
    if args.nt and not large:
        w = w.with_(nt=args.nt)
    nsrc = len(w.sources)
    log(f"[bench] workload {w.name} padded cells {w.padded_cells} sources {nsrc}")
    if args.gradient_sample:
        w = w.with_(nt=args.gradient_sample)
        with emm.Model(w, tile_kz=args.tile_kz, graph_steps=args.graph, tile_x=args.tile_x,
                       tile_rows=args.tile_rows, src_order=args.src_order,
                       nontemporal=args.nontemporal) as m:
            G = m.forward()
            m.gradient(g_bar=G)          # sizes the checkpoint buffers
            m.forward()                  # leaves no checkpoints: the timed call runs its forward
            t = time.perf_counter()
            m.gradient(g_bar=G)
            dt = time.perf_counter() - t
            i = m.info()
        log(f"[bench] gradient sample: {w.name}, {args.gradient_sample} steps, {nsrc} sources, "
            f"forward + gradient {dt * 1e3:.1f} ms, checkpoints every {i['ckpt_outer']} "
            f"(inner {i['ckpt_inner']}), sources per sweep {i['src_group']}")
        return

    t_create = time.perf_counter()
    model = emm.Model(w, profile=1, graph_steps=args.graph, tile_kz=args.tile_kz, fused=args.fused,
                      tile_x=args.tile_x, tile_rows=args.tile_rows, src_order=args.src_order,
                      **({"airwave": args.air_transform} if w.airwave else {}),
                      nontemporal=args.nontemporal)
    create_s = time.perf_counter() - t_create
    wall, acc, info = timed_forwards(model, args.steps, args.warmup, "main")
    model.close()
    nt = info["nt"]
    cells = info["cells"]
    ms_per_step = wall / args.steps * 1e3
    value = cells * nt * nsrc * args.steps / wall / 1e9
    e_avg_s = acc["e_ms"] / acc["e_n"] / 1e3 if acc["e_n"] else float("nan")
    h_avg_s = acc["h_ms"] / acc["h_n"] / 1e3 if acc["h_n"] else float("nan")
    fused = bool(info["fused"])
    kb = kernel_bytes(info, nsrc)
    if fused:
        e_bytes = e_moved = info["leap_bytes"] * nsrc
    else:
        e_bytes, e_moved = kb["e_8d"], kb["e_moved"]
    achieved = e_bytes / e_avg_s / 1e9
    log(f"[bench] nt={nt} wall/step={ms_per_step:.1f} ms device loop/step="
        f"{acc['dev_ms'] / args.steps:.1f} ms e_step avg={e_avg_s * 1e6:.2f} us "
        f"h_step avg={h_avg_s * 1e6:.2f} us tile_kz={info['tile_kz']} tile_x={info['tile_x']} "
        f"tile_rows={info['tile_rows']} src_order={info['src_order']} nontemporal={info['nontemporal']} "
        f"ce_table={info['ce_table']}")
    full_nt = json.load(open(LARGE_GOLDEN))["nt"] if large and os.path.exists(LARGE_GOLDEN) else None
    step_desc = (f"one forward of the {nsrc} sources batched, over a window of {nt} time steps "
                 + (f"(of the {full_nt} of a full run)" if full_nt else "of a full run")
                 if large else "one full forward modelling (nt time steps)")
    out = {
        "metric": "FDTD cell-updates/s (Gcell*step/s) + % HBM peak; batched fwd+grad vs plain fwd",
        "value": value, "unit": "Gcell*step/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (fields), " + ("f32 Kahan-compensated" if w.dft_mode else "f64") + " (DTFT)",
        "data": "synthetic",
        "config": {"workload": w.name, "padded_cells": cells, "time_steps": nt, "rd": w.rd,
                   "sources": nsrc, "receivers": len(w.receivers), "channels": 6,
                   "freqs": [float(f) for f in w.freqs], "step": step_desc,
                   "value_counts": "padded cells x time steps x sources"},
        "roofline": {"bound": "hbm",
                     "kernel": ("leap (E update + H update of one step)") if fused else
                               "e_step (curl H + CPML + J + E update + H-channel DTFT)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if fused else traffic(w.name, "e_step", info, nsrc),
                     "bytes_per_launch": e_bytes, "bytes_moved_per_launch": e_moved,
                     "moved_GBs": e_moved / e_avg_s / 1e9, "avg_launch_us": e_avg_s * 1e6,
                     "launches_timed": acc["e_n"]},
        "interior_gcell_step_per_s": (len(w.x1) * len(w.x2) * len(w.x3)) * nt * nsrc * args.steps / wall / 1e9,
        "device_loop_ms_per_step": acc["dev_ms"] / args.steps,
        "ms_per_step_median": float(sorted(acc["walls"])[len(acc["walls"]) // 2] * 1e3),
        # set-up: emm_create (padded grid, FD tables, dt/eps, device
        # allocation and upload of the model; outside the timed region), and
        # the host share of each forward (acquisition tables, launches,
        # read-back; inside it)
        "setup": {"model_create_s": create_s,
                  "per_forward_host_ms": (wall - acc["dev_ms"] / 1e3) / args.steps * 1e3},
        "launch": {"tile_kz": info["tile_kz"], "tile_x": info["tile_x"], "tile_rows": info["tile_rows"],
                   **({"air_transform": ("hipfft", "direct")[info["air_transform"] - 1]}
                      if info["air_transform"] else {}),
                   "src_order": info["src_order"], "nontemporal": info["nontemporal"],
                   "compact_dt_eps": info["ce_table"], "graph_steps": args.graph},
    }
    if not fused:
        out["h_step"] = {"bytes_per_launch": kb["h"], "avg_launch_us": h_avg_s * 1e6,
                         "achieved_GBs": kb["h"] / h_avg_s / 1e9,
                         "frac": kb["h"] / h_avg_s / 1e9 / HBM_PEAK_GBS,
                         "traffic": traffic(w.name, "h_step", info, nsrc)}
    # the counter traffic per launch as a rate against both peaks
    tr = out["roofline"]["traffic"]
    if tr:
        out["roofline"]["traffic_GBs"] = tr / e_avg_s / 1e9
        out["roofline"]["traffic_frac"] = tr / e_avg_s / 1e9 / HBM_PEAK_GBS
    if stream_ref:
        out["stream_reference"] = dict(stream_ref)
        out["stream_reference"]["e_step_frac_of_it"] = achieved / stream_ref["GBs"]
        if tr:
            out["stream_reference"]["e_step_traffic_frac_of_it"] = tr / e_avg_s / 1e9 / stream_ref["GBs"]
    if large and not args.quick:
        log("[bench] batched forward + gradient legs")
        out["batched"] = large_batched(emm, w, nt, ms_per_step / 1e3)
        if os.path.exists(LARGE_GOLDEN):
            log("[bench] accuracy against the stored FP64 oracle result (full step count)")
            out["accuracy"] = accuracy_vs_golden(emm, LARGE_GOLDEN, configs.large_marine(rd=4, nsrc=8),
                                                 "large")
        if os.path.exists(PLAIN_GOLDEN):
            log("[bench] 48^3 plain forward against the stored oracle result and the analytic dipole")
            out["accuracy_48cube"] = plain_accuracy(emm)
        log("[bench] towline of 16 sources on the 48^3 model")
        out["towline_48cube"] = small_towline(emm)
        log("[bench] marine (cache-resident) leg")
        out["marine"] = marine_leg(emm, 3)
    if args.multi_model:
        log("[bench] multi-model comparison")
        out["multi_model"] = multi_model_comparison(emm, args.graph or 64)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps if large else 200,
                                           args.cpu_steps_one if large else 20)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
