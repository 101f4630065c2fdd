"""Benchmark of the Coulomb-process Monte Carlo step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg5]

Prints one JSON line: pair evaluations per second over the K timed steps
(the pair tests of all processes, summed; inputs resident in HBM), the FP32
form against the plain FP64 form on the same cells, the HBM roofline of the
pair-test kernel (algorithmic bytes per launch over its duration, from HIP
events that the launches of K further steps stamp at kernel start and end)
and the FP64 CPU oracle timed on a bounded sample of the same workload.

python bench.py --copy-calibration runs only a device-to-device copy of
known size: the counter runs that measure the kernel's HBM traffic read the
same counters on it to scale them.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pair evaluations/sec + % HBM peak; FP32-batched vs FP64-plain at 1e-5 rel err"
COUNTERS = {"cfg2": os.path.join(ROOT, "profiles", "k_pass_bh_cfg2_counters.txt"),
            "cfg5": os.path.join(ROOT, "profiles", "k_stream_cfg5_counters.txt")}
CFG5_SAMPLE = 1024             # seeded cells of cfg5 the oracle runs (global cell ids)
COPY_BYTES = 1 << 30
HIP_EVENT_DISABLE_SYSTEM_FENCE = 0x20000000

WORKLOADS = {
    "cfg5": ("Foil-transport scale, Bremsstrahlung -> Bethe-Heitler chain: 131072 cells x (4096 electrons "
             "+ 4096 Au ions), Z* = 5, n_i = 5.9e22 cm^-3, T_e = 1 eV, electrons Maxwell-Juttner T = 5 MeV "
             "(isotropic, W_e = 1.5e19 cm^-3/4096), photon/e-/e+ slabs 2 x 4096 per cell, dt = 0.05 fs; "
             "generated in HBM"),
    "cfg2": ("Bethe-Heitler pairs, FP32 tables + FP64 tallies: 4096 cells x (1024 photons + "
             "1024 Au ions), Z* ~ U[0,79] per cell, n_i = 5.9e22 cm^-3, T_e log-uniform "
             "10 eV-10 keV, photon energy 1.022 MeV + Exp(5 MeV), log-normal weights, dt = 0.1 fs"),
    "cfg1": ("Plain FP64 Bremsstrahlung: 64 cells x (256 electrons + 256 Cu ions), Z* = 10, "
             "T_e = 100 eV, 1-100 MeV log-uniform, dt = 0.1 fs"),
    "cfg3": ("Batched uneven cells, all three processes: 16384 cells, power-law (alpha = 1.5) "
             "counts on [16, 8192] per species, Au, dt = 0.1 fs"),
}


def source_digest():
    """SHA-256 of the HIP sources: stored counter figures are used only
    while the kernels they were taken on are unchanged."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1907_02814_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


class HipEvents:
    """Raw hipEvent_t handles (the library records them on its launch
    stream; torch's events only see torch's current stream)."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]

    def create(self, n):
        out = []
        for _ in range(n):
            e = ctypes.c_void_p()
            # timing only: no system-scope fence (cache writeback and
            # invalidation) when the event completes
            rc = self.lib.hipEventCreateWithFlags(ctypes.byref(e), HIP_EVENT_DISABLE_SYSTEM_FENCE)
            if rc != 0:
                raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
            out.append(e.value)
        return out

    def record(self, e, stream):
        rc = self.lib.hipEventRecord(ctypes.c_void_p(e), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        rc = self.lib.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def destroy(self, evs):
        for e in evs:
            self.lib.hipEventDestroy(ctypes.c_void_p(e))


def make_workload(name, W):
    """The workload in device memory: cfg5 is generated there (125 GB),
    the others on the host and copied."""
    if name == "cfg5":
        return W.cfg5_device("cuda:0")
    return getattr(W, name)().to_torch("cuda:0")


def count_evals(make, precision, steps, warmup, schedule, seed=1):
    """Pair evaluations and events of steps warmup .. warmup + K - 1, run
    eagerly on a fresh copy of the workload with a tally row per step.  A
    step's results do not depend on the launch shape or on graph replay, so
    these are the counts of the graph-replayed steps of the same numbers."""
    import torch
    import paper_1907_02814_amd as cmc
    g = make()
    tab = cmc.build_tables(g.Z)
    st = cmc.StepState(tab, g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po, dt=g.dt,
                       seed=seed, processes=g.processes, precision=precision, schedule=schedule)
    n = g.cells["Zstar"].numel()
    rows = torch.zeros((steps, n, len(cmc.I_NAMES)), dtype=torch.int64, device="cuda:0")
    for s in range(warmup):
        st.step(s)
    for i in range(steps):
        st.set_tallies(ti=rows[i])
        st.step(warmup + i)
    torch.cuda.synchronize()
    evals = int(rows[:, :, 0:3].sum().item())
    events = rows[:, :, 3:6].sum((0, 1)).tolist()
    del st, g, rows
    torch.cuda.empty_cache()
    return evals, events


def run_gpu(make, precision, steps, warmup, schedule, seed=1, graph=False):
    """K timed steps of a fresh copy of the workload (make() builds it in
    device memory) whose pair-test launches stamp HIP events on their stream
    (the first launch at its start, a record after the last): the wall time
    of the K steps gives the throughput, the events the kernel durations of
    the same steps.  Each timed step writes its integer tallies to a row of
    its own (the pass kernels count the pairs they test), so the pair
    evaluations of the timed steps are summed afterwards, outside the timed
    region.  graph: the timed steps are replays of one captured step (its
    tallies in one buffer; the counts come from count_evals), and W + K
    eager steps stamped after them give the kernel durations (of the last
    K: after the host's pause the device runs its first steps slower)."""
    import torch
    import paper_1907_02814_amd as cmc
    g = make()
    tab = cmc.build_tables(g.Z)
    st = cmc.StepState(tab, g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po, dt=g.dt,
                       seed=seed, processes=g.processes, precision=precision, schedule=schedule)
    n = g.cells["Zstar"].numel()
    stream = torch.cuda.current_stream()
    H = HipEvents()
    evs = H.create(2 * (warmup + steps))
    for s in range(warmup):
        st.step(s, stream)
    torch.cuda.synchronize()
    # the live photons before the first and after the last measured step
    # (their mean over the steps, by linear growth, for the algorithmic bytes)
    ng0 = int(g.photons["count"].sum().item())
    if graph:
        gr, counter = st.graph(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            gr.replay()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st.use_counter(None)
        del gr, counter
        evals, events = None, None
        ng0 = int(g.photons["count"].sum().item())
        for i in range(warmup + steps):
            st.step(warmup + steps + i, stream, events=(evs[2 * i], evs[2 * i + 1]))
        torch.cuda.synchronize()
        pass_ms = [H.elapsed_ms(evs[2 * i], evs[2 * i + 1]) for i in range(warmup, warmup + steps)]
    else:
        rows = torch.zeros((steps, n, len(cmc.I_NAMES)), dtype=torch.int64, device="cuda:0")
        t0 = time.perf_counter()
        for i in range(steps):
            st.set_tallies(ti=rows[i])
            st.step(warmup + i, stream, events=(evs[2 * i], evs[2 * i + 1]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st.set_tallies(ti=None)
        pass_ms = [H.elapsed_ms(evs[2 * i], evs[2 * i + 1]) for i in range(steps)]
        evals = int(rows[:, :, 0:3].sum().item())
        events = rows[:, :, 3:6].sum((0, 1)).tolist()
        del rows
    ng1 = int(g.photons["count"].sum().item())
    H.destroy(evs)
    status = int(st.status.item())
    alg = algorithmic_bytes_dev(g, ng0 + (ng1 - ng0) * (steps - 1) / (2 * steps))
    step_b = alg + g.cells["Zstar"].numel() * (24 + 12 * 8 + 10 * 8)
    del st, g
    torch.cuda.empty_cache()
    if graph:
        evals, events = count_evals(make, precision, steps, warmup, schedule, seed)
    return {"wall_s": wall, "pass_ms": pass_ms, "evals": evals, "status": status,
            "events": events, "alg_bytes": alg, "step_bytes": step_b}


def algorithmic_bytes_dev(g, ng):
    """Bytes the pair tests of one step must move, for a device workload
    with ng live photons (the mean over the measured steps): one read of
    every live mobile record per pass (px, py, pz, w = 32 B), one read of
    each ion weight per step (8 B: both passes use the same ion sums, which
    the photon-ion pass takes from the electron-ion pass in every cell
    that has electrons) and the per-cell tallies the passes write (pairs
    and n_ab: 16 B per pass).  The whole step adds the cell parameters
    (24 B) and the full tally rows (12 * 8 + 10 * 8 B) per cell."""
    ne_c = g.electrons["off"][1:] - g.electrons["off"][:-1]
    ni_c = g.ions["off"][1:] - g.ions["off"][:-1]
    ne, ni = int(ne_c.sum().item()), int(ni_c.sum().item())
    n = g.cells["Zstar"].numel()
    ei, gi = bool(g.processes & 5), bool(g.processes & 2)
    b = 0
    if ei:
        b += 32 * ne + 8 * ni + 16 * n
    if gi:
        ions_again = ni if not ei else int(ni_c[ne_c == 0].sum().item())
        b += 32 * ng + 8 * ions_again + 16 * n
    return b


def stored_traffic(workload):
    """HBM bytes per step of the pass kernels from the stored counter runs
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a copy of
    known size), or None when absent or taken on other kernel sources."""
    path = COUNTERS.get(workload)
    if path is None:
        return None
    try:
        with open(path) as fh:
            kv = dict(l.split(":", 1) for l in fh if ":" in l and not l.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("source_sha256") != source_digest():
            return None
        fetch = float(kv["pass FETCH_SIZE KiB/dispatch"]) * float(kv["copy read scale"])
        write = float(kv["pass WRITE_SIZE KiB/dispatch"]) * float(kv["copy write scale"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def _oracle_rate(wl, cores, budget_s, seed):
    from oracle import oracle as O
    tab = O.tables(wl.Z)
    ref = wl.copy()
    evals = 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        ti, td, st = O.collide_step(tab, ref.cells, ref.electrons, ref.photons, ref.ions, ref.new_el,
                                    ref.new_po, wl.dt, seed, steps, wl.processes, nthreads=cores)
        evals += int(ti[:, 0:3].sum())
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 1000:
            break
    return evals / el, steps, evals, el


def cpu_baseline(wl, what, budget_s=12.0, seed=1):
    """The FP64 oracle on the host cores, on `wl` (a host workload: the
    whole workload, or the seeded sample of cfg5's cells with their global
    ids, so that it draws the numbers the GPU run draws there), stepping
    from step 0 for about budget_s; then on one core for a third of that."""
    cores = len(os.sched_getaffinity(0))
    v, steps, evals, el = _oracle_rate(wl, cores, budget_s, seed)
    v1, steps1, evals1, el1 = _oracle_rate(wl, 1, budget_s / 3.0, seed)
    return {"value": v, "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} step(s) of {what}, {evals} pair evaluations in {el:.2f} s "
                      f"(FP64, OpenMP over cells)",
            "one_core": {"value": v1, "steps": steps1, "seconds": el1}}


YIELD_WORKLOAD = ("cfg4: expected yield and its adjoint, 1024 cells x 4096 electrons (FP64 momenta), "
                  "gamma log-uniform 2-1000, Cu, Z* ~ U[1,29], n_e log-uniform 1e21-1e24 cm^-3, "
                  "T_e log-uniform 10 eV-10 keV, dt = 0.1 fs")


def yield_bytes(n_cells, n_el):
    """Algorithmic bytes of one call: forward reads px, py, pz, w (32 B per
    electron) and the cell parameters (24 B), writes Y (8 B per cell); the
    adjoint reads the same and gY and writes gpx, gpy, gpz (24 B per
    electron) and three cell gradients.  (It is timed without the optional
    gradient with respect to the weights.)"""
    fwd = 32 * n_el + 32 * n_cells
    bwd = 56 * n_el + 56 * n_cells
    return fwd, bwd


def run_yield(calls=20, seed_cells=64, cpu=True):
    """Expected yield (cfg4), forward and adjoint, both forms: the average
    time per call of `calls` back-to-back calls between two HIP events on
    the calls' stream, and the FP64 oracle on the first `seed_cells` cells."""
    import torch
    import paper_1907_02814_amd as cmc
    from paper_1907_02814_amd import workloads as W
    y = W.cfg4()
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in y.items() if isinstance(v, np.ndarray)}
    n_cells, n_el = len(y["Zstar"]), len(y["px"])
    tab = cmc.build_tables(y["Z"])
    gY = torch.ones(n_cells, dtype=torch.float64, device=dev)
    H = HipEvents()
    stream = torch.cuda.current_stream()
    args = (t["Zstar"], t["n_e"], t["T_e"], t["off"], t["px"], t["py"], t["pz"], t["w"], y["dt"])
    fwd_b, bwd_b = yield_bytes(n_cells, n_el)
    out = {"workload": YIELD_WORKLOAD, "electrons": n_el}
    for name, prec in (("fp32", cmc.FP32), ("fp64", cmc.FP64)):
        row = {}
        for kind, fn, nbytes in (("forward", lambda: cmc.expected_yield(tab, *args, precision=prec), fwd_b),
                                 ("adjoint", lambda: cmc.expected_yield_backward(tab, *args, gY, precision=prec,
                                                                                 weight_grad=False), bwd_b)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = H.create(2)
            H.record(e0, stream)
            for _ in range(calls):
                fn()
            H.record(e1, stream)
            torch.cuda.synchronize()
            ms = H.elapsed_ms(e0, e1) / calls
            H.destroy([e0, e1])
            row[kind] = {"ms_per_call": ms, "electron_evals_per_s": n_el / (ms * 1e-3),
                         "alg_bytes": nbytes, "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[name] = row
    if not cpu:
        return out
    # the oracle on a bounded sample of the same cells
    from oracle import oracle as O
    otab = O.tables(y["Z"])
    k = seed_cells
    e = int(y["off"][k])
    sl = (y["Zstar"][:k], y["n_e"][:k], y["T_e"][:k], y["off"][:k + 1], y["px"][:e], y["py"][:e],
          y["pz"][:e], y["w"][:e], y["dt"])
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    O.expected_yield(otab, *sl, nthreads=cores)
    t1 = time.perf_counter()
    O.expected_yield_backward(otab, *sl, np.ones(k), nthreads=cores)
    t2 = time.perf_counter()
    out["cpu_baseline"] = {"forward_electron_evals_per_s": e / (t1 - t0),
                           "adjoint_electron_evals_per_s": e / (t2 - t1), "cores": cores, "kind": "oracle",
                           "sample": f"the first {k} cells ({e} electrons), forward and adjoint once each (FP64)"}
    return out


def measured_hbm():
    """Device bandwidth measured on this GPU beside the published 8 TB/s:
    a 1 GiB device-to-device copy (read + write bytes) and a read-only sum
    of 2 GiB of doubles (torch's kernels), best of 5."""
    import torch
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    r = torch.empty(2 * COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").uniform_()
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * COPY_BYTES), ("read", lambda: r.sum(), 2 * COPY_BYTES)):
        fn()
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[f"{name}_GBs"] = nbytes / (best * 1e-3) / 1e9
    del a, b, r
    torch.cuda.empty_cache()
    return out


def copy_calibration():
    import torch
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "dispatches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default="auto", choices=["auto", "group", "wave", "hybrid", "cell", "queue", "split"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-yield", action="store_true", help="skip the expected-yield measurement")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of a captured step (default for cfg3, the batched form)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of known size (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); cells are independent within a step, so the "
              "path would shard by contiguous cell ranges with no exchange; the library runs "
              "and this benchmark measures one GPU's share", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    import paper_1907_02814_amd as cmc
    from paper_1907_02814_amd import workloads as W
    sched = {"auto": cmc.SCHED_AUTO, "group": cmc.SCHED_GROUP, "wave": cmc.SCHED_WAVE,
             "hybrid": cmc.SCHED_HYBRID, "cell": cmc.SCHED_CELL, "queue": cmc.SCHED_QUEUE,
             "split": cmc.SCHED_SPLIT}[a.schedule]
    print(f"[bench] {a.workload}", file=sys.stderr, flush=True)
    make = lambda: make_workload(a.workload, W)
    if a.workload == "cfg5":
        # the oracle's sample: seeded cells of the same initial state
        g0 = make()
        sample = np.sort(np.random.default_rng(1005).choice(g0.cells["Zstar"].numel(), CFG5_SAMPLE, replace=False))
        host_wl = g0.host_subset(sample)
        what = f"{CFG5_SAMPLE} seeded cells of the same workload (global cell ids)"
        del g0
        import torch
        torch.cuda.empty_cache()
    else:
        host_wl = getattr(W, a.workload)()
        what = f"all {host_wl.n_cells} cells of the same workload"
    graph = a.graph or a.workload == "cfg3"
    fp32 = run_gpu(make, cmc.FP32, a.steps, a.warmup, sched, graph=graph)
    print(f"[bench] fp32 done: {fp32['wall_s'] * 1e3 / a.steps:.3f} ms/step", file=sys.stderr, flush=True)
    fp64 = None if a.no_fp64 else run_gpu(make, cmc.FP64, a.steps, a.warmup, sched, graph=graph)
    if fp64:
        print(f"[bench] fp64 done: {fp64['wall_s'] * 1e3 / a.steps:.3f} ms/step", file=sys.stderr, flush=True)
    kavg = float(np.mean(fp32["pass_ms"]))
    alg = fp32["alg_bytes"]
    achieved = alg / (kavg * 1e-3) / 1e9
    ms = fp32["wall_s"] * 1e3 / a.steps
    value = fp32["evals"] / fp32["wall_s"]
    traffic = stored_traffic(a.workload) if a.schedule == "auto" else None
    # the pair-test kernels of the step: the stream kernel takes the cells
    # whose ions are at rest and whose electrons pair once (both passes of
    # every cfg5 cell), the pass kernel the rest
    kname = "k_stream<float> + k_pass<float> (the cells k_stream leaves)"
    out = {
        "metric": METRIC, "value": value, "unit": "pair-evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32 lookups + fp64 probability/tallies",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS[a.workload]}", "cells": int(host_wl.n_cells if a.workload != "cfg5" else 131072),
                   "pairs_per_step": fp32["evals"] // a.steps, "schedule": a.schedule, "graph_replay": graph,
                   "parallelism": "single GPU, cells"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "kernel_ms": kavg, "alg_bytes_per_launch": alg},
        "step_hbm_frac": fp32["step_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "status": fp32["status"],
        "events_per_step": [e / a.steps for e in fp32["events"]],
    }
    if fp64:
        v64 = fp64["evals"] / fp64["wall_s"]
        k64 = float(np.mean(fp64["pass_ms"]))
        out["fp64_plain"] = {"value": v64, "ms_per_step": fp64["wall_s"] * 1e3 / a.steps,
                             "kernel_ms": k64, "hbm_frac": fp64["alg_bytes"] / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "step_hbm_frac": fp64["step_bytes"] / (fp64["wall_s"] / a.steps) / 1e9 / HBM_PEAK_GBS}
        out["fp32_speedup_vs_fp64"] = value / v64
    out["roofline"]["measured_peak"] = measured_hbm()
    if not a.no_yield:
        print("[bench] expected yield", file=sys.stderr, flush=True)
        out["expected_yield"] = run_yield(cpu=not a.no_cpu)
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(host_wl, what)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
