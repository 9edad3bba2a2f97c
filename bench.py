#!/usr/bin/env python3
"""Benchmark of the exponential-midpoint / Krylov time stepper on one MI355X.

Workload (one "step" = one midpoint step: every Lanczos iteration's
matrix-free H*v, the FP64 recurrence and small exponential, the combine, and
the fused observables): 12-site 3x4 periodic cluster, t = 1, U = 8, half
filling 6/6 (dim 853,776), field along x with A0 drawn from the seeded
uniform [0.2, 1.0], omega = 8, sigma = 0.5, t0 = 2.5; dt = 0.005, Krylov
tol 1e-10, m_max 30; single complex128 vector.  The ground state of H(0) is
advanced untimed to the start of a window of K steps centred on the pulse
(t0), so the timed steps are the pulse regime whatever K is.  All inputs
synthetic and resident in HBM before timing.

Prints one JSON line (metric, value = midpoint steps/s, roofline of the H*v
kernel measured with HIP events over the timed region, CPU-oracle baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H·v HBM GB/s + midpoint steps/s at 12 sites: mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0
# Fused Lanczos iteration of the 12-site complex128 vector (update of u_j +
# two-pass H*v + epilogue): row pass without up hops that also forms u_j, and
# the column pass; 20 padded hop slots
DOMINANT_KERNELS = ("k_apply<double, 1, 1, 20, 256, false, true, false>", "k_colpass<double, 1, 20, 1024, true, false, 4>")
# Speculative iterations enqueued past a step's Krylov decision exit at once,
# and the column pass of a step's last fused iteration skips its apply; a
# dispatch below this fraction of the kernel's 90th percentile (time or bytes;
# more than a tenth of the dispatches do the work, and slow outliers are
# rarer) is counted as such and left out of the per-launch figures.
EARLY_EXIT_FRACTION = 0.5


def early_exit_cut(vals) -> float:
    v = sorted(vals)
    return EARLY_EXIT_FRACTION * v[(9 * (len(v) - 1)) // 10]
UNIT_BYTES = 4 * 853776 * 16  # read w_{j-1}, u_{j-1}; write u_j, y
COUNTERS_FILE = os.path.join(ROOT, "profiles", "lanczos_iter_c128_cluster3x4_counters.txt")
STATS_FILE = os.path.join(ROOT, "profiles", "bench_cluster3x4_c128_kernel_stats.txt")
KERNEL_SOURCES = ("paper_2005_13498_amd/csrc/apply_impl.h", "paper_2005_13498_amd/csrc/kernels_common.h",
                  "paper_2005_13498_amd/csrc/apply_c128.hip", "paper_2005_13498_amd/csrc/kernels.h",
                  "paper_2005_13498_amd/csrc/kernels.hip")
COPY_BYTES = 256 << 20  # calibration copy: bytes read (and written) per launch
PROFILE_PERIOD = 32     # HIP events on every 32nd fused iteration (an event-carrying dispatch costs a few us)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None if there is none or the kernel sources changed since."""
    try:
        kv = {}
        with open(COUNTERS_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def traced_pair_us():
    """Average kernel time (us) of a working fused iteration in the committed
    rocprofv3 trace summary of this workload, or None if there is none or the
    kernel sources changed since."""
    try:
        kv = {}
        with open(STATS_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["fused_iteration_avg_us (both kernels, working dispatches)"])
    except (OSError, KeyError, ValueError):
        return None


def trace_figure(bytes_per: float):
    """The same kernel pair as timed by the committed rocprofv3 trace (kernel
    execution only; HIP events also count their own timestamping), or None."""
    us = traced_pair_us()
    if not us:
        return None
    gbs = bytes_per / (us * 1e-6) / 1e9
    return {"avg_launch_us": us, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
            "source": os.path.relpath(STATS_FILE, ROOT)}


def _rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def copy_calibration() -> None:
    """A plain elementwise kernel over COPY_BYTES (read and written), whose
    counters scale the H*v kernels' to bytes."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


# Counter summaries: the fused Lanczos pair of each workload, its title and its
# algorithmic bytes per iteration (4 N s: read w_{j-1}, u_{j-1}; write u_j, y)
COUNTER_CASES = {
    "cluster3x4": (DOMINANT_KERNELS,
                   ["# HBM traffic of one fused Lanczos iteration (complex128, 12-site 3x4, dim 853776):"], UNIT_BYTES),
    "ring14": (("k_apply<double, 1, 1, 16, 1024, false, true, false>", "k_colpass<double, 1, 16, 1024, true, true, 2>"),
               ["# HBM traffic of one fused Lanczos iteration (complex128, 14-site ring 7/7, dim 11778624,",
                "# vectors far beyond the Infinity Cache; column pass staging one copy of 2 tile columns):"],
               4 * 11778624 * 16),
}


def summarize_counters(fetch_dir: str, write_dir: str, out: str, command: str, case: str = "cluster3x4") -> None:
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the H*v kernels and of the
    calibration copy, scaled by the copy's known bytes, written as text."""
    import statistics
    kernels, title, unit_bytes = COUNTER_CASES[case]

    def per_kernel(d, counter):
        vals = {}
        for r in _rows(_find(d, "counter_collection.csv")):
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    lines = title + [
             "# u_j = w_{j-1} - alpha s u_{j-1} and H u_j with the Lanczos epilogue, as the row pass",
             "# and the column pass of the two-pass apply, per dispatch, summed",
             f"# command: {command}",
             "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by what it reads for a",
             f"# copy of {COPY_BYTES} bytes (torch elementwise neg, bench.py --copy-calibration)."]
    res = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        v = per_kernel(d, counter)
        cp = [k for k in v if "neg_kernel" in k]
        if not cp:
            raise SystemExit(f"{counter}: copy kernel missing: {sorted(v)[:8]}")
        cpk = max(statistics.mean(v[k]) for k in cp)
        factor = COPY_BYTES / (cpk * 1024.0)
        kib = 0.0
        for want in kernels:
            hit = [k for k in v if want in k]
            if not hit:
                raise SystemExit(f"{counter}: kernel {want} missing: {sorted(v)[:8]}")
            allv = v[hit[0]]
            work = [x for x in allv if x >= early_exit_cut(allv)]
            m = statistics.mean(work)
            kib += m
            lines += [f"{counter}_kernel: {hit[0]}", f"{counter}_dispatches: {len(work)} "
                      f"(plus {len(allv) - len(work)} early exits or skipped applies past the Krylov decision, left out)",
                      f"{counter}_kib_per_dispatch: {m:.1f}"]
        res[name] = kib * 1024.0 * factor
        lines += [f"{counter}_copy_kib_per_dispatch: {cpk:.1f}", f"{counter}_copy_scale: {factor:.4f}"]
    lines += [f"hbm_fetch_bytes_per_launch: {res['fetch']:.0f}", f"hbm_write_bytes_per_launch: {res['write']:.0f}",
              f"hbm_bytes_per_launch: {res['fetch'] + res['write']:.0f}",
              f"algorithmic_bytes_per_launch: {unit_bytes}",
              f"kernel_source_sha256_16: {kernel_source_hash()}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(trace_dir: str, out: str, command: str, top: int = 16, note: str = "") -> None:
    """Top kernels of a --kernel-trace --stats run as text (and the fused
    iteration's split when the trace has it)."""
    rows = _rows(_find(trace_dir, "kernel_stats.csv"))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}"]
    lines += [f"# {x}" for x in note.split("|") if x]
    lines += [f"{'calls':>8} {'avg_us':>10} {'total_ms':>10} {'pct':>6}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):>8} {float(r['AverageNs']) / 1e3:>10.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:>10.2f} {float(r['Percentage']):>6.2f}  {r['Name'][:150]}")
    try:
        trace = _rows(_find(trace_dir, "kernel_trace.csv"))
    except SystemExit:
        trace = []
    if trace and any(want in r["Kernel_Name"] for r in trace for want in DOMINANT_KERNELS):
        lines += ["", "# fused Lanczos iteration (the roofline kernel pair), from the per-dispatch trace:",
                  f"# dispatches under {EARLY_EXIT_FRACTION} x the kernel's 90th percentile are speculative launches past",
                  "# the Krylov decision (they exit at once) or the skipped column pass of a step's last iteration,",
                  "# and are left out, as in bench.py's event timing"]
        tot = 0.0
        for want in DOMINANT_KERNELS:
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
                 if want in r["Kernel_Name"]]
            if not d:
                continue
            cut = early_exit_cut(d)
            work = [x for x in d if x >= cut]
            early = [x for x in d if x < cut]
            avg = sum(work) / len(work)
            tot += avg
            lines.append(f"{want}: working {len(work)} avg_us {avg:.2f}; early exits {len(early)}"
                         + (f" avg_us {sum(early) / len(early):.2f}" if early else ""))
        lines.append(f"fused_iteration_avg_us (both kernels, working dispatches): {tot:.2f}")
        lines.append(f"kernel_source_sha256_16: {kernel_source_hash()}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_baseline(seconds: float, member: int = -1) -> dict:
    """Oracle timing on the host (run in a single-threaded child process).
    member >= 0: only the midpoint steps of that member of the 8-pulse batch
    (its A0 draw), for the all-cores figure."""
    import numpy as np
    from synth import workloads, random_state, PulseParams
    from oracle import HubbardOracle, pulse_A, krylov_step_alg6

    w = workloads()["cluster3x4"]
    if member >= 0:
        p0 = w.pulse
        w = w.__class__(**{**w.__dict__, "pulse": PulseParams(p0.kind, w.extra["A0_batch"][member], p0.omega,
                                                                  p0.t0, p0.sigma)})
    ham = HubbardOracle(w.lattice, w.U, w.n_up, w.n_dn)
    hn = ham.norm_inf()
    import scipy.sparse.linalg as spla
    # start: the oracle's own ground state of H(0) (loose tolerance: setup only)
    A0 = pulse_A(w.pulse, 0.0)
    H0 = ham.H(A0)
    _, vecs = spla.eigsh(H0, k=1, which="SA", tol=1e-8, v0=random_state(ham.dim, seed=3)[0])
    v = vecs[:, 0].astype(np.complex128)
    # timed: literal Alg. 6 midpoint steps, same tolerance and step as the GPU run
    t = 0.0
    steps = 0
    ms = []
    hv = 0
    t_start = time.perf_counter()
    while True:
        A = pulse_A(w.pulse, t + 0.5 * w.dt)
        H = ham.H(A)

        def apply(x):
            nonlocal hv
            hv += 1
            return H @ x

        v, info = krylov_step_alg6(apply, v, w.dt, w.m_max, w.tol, hn)
        ms.append(info["m"])
        steps += 1
        t += w.dt
        el = time.perf_counter() - t_start
        if el >= seconds:
            break
    if member >= 0:
        return {"member": member, "steps_per_s": steps / el, "steps": steps}
    # the oracle's H*v alone (m-independent): scipy CSR at A = 0.5, 1 thread
    H = ham.H(0.5)
    x = random_state(ham.dim, seed=1)[0]
    H @ x
    t1 = time.perf_counter()
    nrep = 10
    for _ in range(nrep):
        H @ x
    hv_ms = (time.perf_counter() - t1) / nrep * 1e3
    # the latency case (8-site ring) on the oracle: literal Alg. 6 steps/s
    w8 = workloads()["ring8"]
    h8 = HubbardOracle(w8.lattice, w8.U, w8.n_up, w8.n_dn)
    hn8 = h8.norm_inf()
    _, vecs8 = spla.eigsh(h8.H(pulse_A(w8.pulse, 0.0)), k=1, which="SA", tol=1e-10,
                          v0=random_state(h8.dim, seed=3)[0])
    v8 = vecs8[:, 0].astype(np.complex128)
    t8, n8 = 0.0, 0
    t2 = time.perf_counter()
    while n8 < w8.n_steps and time.perf_counter() - t2 < 5.0:
        H8 = h8.H(pulse_A(w8.pulse, t8 + 0.5 * w8.dt))
        v8, _ = krylov_step_alg6(lambda z: H8 @ z, v8, w8.dt, w8.m_max, w8.tol, hn8)
        t8 += w8.dt
        n8 += 1
    ring8_sps = n8 / (time.perf_counter() - t2)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": steps / el, "unit": "midpoint steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} literal Alg.6 midpoint steps of the 12-site 3x4 workload from the "
                      f"oracle ground state (scipy CSR complex128, tol {w.tol:g}, dt {w.dt}, mean m "
                      f"{float(np.mean(ms)):.2f}, {hv} H*v in {el:.1f} s, 1 thread)",
            "hv_ms_1core": hv_ms, "hv_gbps_algorithmic_1core": 2 * ham.dim * 16 / (hv_ms * 1e-3) / 1e9,
            "ring8_steps_per_s_1core": ring8_sps, "ring8_steps_timed": n8,
            "host_cpus": os.cpu_count(), "host_cpu_model": model}


def plan_label(hub, B, prec: int, nvec: int, propagate: bool) -> str:
    """What the library runs for nvec vectors: group sizes and their kernels."""
    names = {0: "one-pass kernel", 1: "two-pass single-vector kernels", 2: "two-pass block kernels"}
    plan = hub.hub_get_plan(B.handle, prec, nvec, propagate)
    parts = {}
    for g, k in plan:
        parts.setdefault((g, k), 0)
        parts[(g, k)] += 1
    return "; ".join(f"{c} group(s) of {g} on the {names[k]}" for (g, k), c in sorted(parts.items()))


def tuned_run(hub, B, prec: int, pulses, t_start: float, dt: float, steps: int, opts, v):
    """The same propagation under the committed tuning table's plan for this
    sector (measured with hub_tune on the GPU): (entry, plan label, seconds,
    obs) or None when the table has no entry for this sector and GPU."""
    import torch
    from paper_2005_13498_amd import tuning

    tab = tuning.load()
    ent = tab.get(tuning.device_name(), {}).get(tuning.key(B, prec))
    if ent is None:
        return None
    hub.hub_set_tuning(B.handle, prec, ent)
    try:
        label = plan_label(hub, B, prec, len(pulses), True)
        hub.hub_propagate(B.handle, pulses, t_start, dt, 2, opts, v.clone(), want_obs=False)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, o, _ = hub.hub_propagate(B.handle, pulses, t_start, dt, steps, opts, v)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        hub.hub_set_tuning(B.handle, prec, None)
    return ent, label, el, o


def batched_variants(hub, B, v0, t_start: float, w, steps: int) -> dict:
    """Mixed precision and batching at 12 sites: the same ground state under
    8 pulse amplitudes (the seeded A0 draws), propagated by one hub_propagate
    call with 8 members in complex64 (FP64 Lanczos scalars; at this size two
    interleaved blocks of 4 on the two-pass block kernels) and in complex128
    (single vectors on the fused two-pass kernels, on concurrent lanes);
    member-steps/s of both (timed without apply timing, which would keep the
    lanes sequential), the fused iteration's kernel time and GB/s from a
    separate sequential run with apply timing, and the complex64 errors in
    d(t), E(t) against the complex128 batch (max over members and sample
    times)."""
    import numpy as np
    import torch
    from synth import PulseParams

    pulses = [PulseParams(0, a, w.pulse.omega, w.pulse.t0, w.pulse.sigma) for a in w.extra["A0_batch"]]
    nv = len(pulses)
    opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
    res = {}
    obs = {}
    for name, dtype, prec_bytes in (("c64_batch8", torch.complex64, 8), ("c128_batch8", torch.complex128, 16)):
        v = v0.to(dtype).repeat(nv).contiguous()
        hub.hub_propagate(B.handle, pulses, t_start, w.dt, 5, opts, v, want_obs=False)  # warm-up
        v = v0.to(dtype).repeat(nv).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, o, log = hub.hub_propagate(B.handle, pulses, t_start, w.dt, steps, opts, v)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # kernel time of the fused iteration: a shorter sequential run with apply timing
        hub.hub_profile_enable(B.handle, PROFILE_PERIOD // 4)
        hub.hub_profile_read(B.handle)
        hub.hub_propagate(B.handle, pulses, t_start, w.dt, max(50, steps // 10), opts,
                          v0.to(dtype).repeat(nv).contiguous(), want_obs=False)
        launches, kms, bpl = hub.hub_profile_read(B.handle)
        hub.hub_profile_enable(B.handle, False)
        us = kms / max(launches, 1) * 1e3
        res[name] = {"kernels": plan_label(hub, B, hub.HUB_C128 if dtype == torch.complex128 else hub.HUB_C64, nv,
                                           True),
                     "member_steps_per_s": nv * steps / el, "ms_per_step": el / steps * 1e3,
                     "timed_avg_launch_us": us, "timed_gbps": bpl / (us * 1e-6) / 1e9 if launches else 0.0,
                     "timed_bytes_per_launch": bpl, "mean_krylov_m": float(np.mean(log[:, :, 0]))}
        obs[name] = o
        print(f"[bench] {name}: {nv * steps / el:.0f} member-steps/s, H*v {us:.1f} us", file=sys.stderr, flush=True)
    d64, d128 = obs["c64_batch8"][:, :, 3], obs["c128_batch8"][:, :, 3]
    e64, e128 = obs["c64_batch8"][:, :, 2], obs["c128_batch8"][:, :, 2]
    res["c64_vs_c128"] = {"max_abs_docc_err": float(np.max(np.abs(d64 - d128))),
                          "max_abs_energy_per_site_err": float(np.max(np.abs(e64 - e128))),
                          "max_abs_norm_drift": float(np.max(np.abs(obs["c64_batch8"][:, :, 1] - 1.0)))}
    tr = tuned_run(hub, B, hub.HUB_C64, pulses, t_start, w.dt, steps, opts, v0.to(torch.complex64).repeat(nv).contiguous())
    if tr is not None:
        ent, label, el, o = tr
        res["c64_batch8_tuned"] = {"kernels": label, "prop_group": ent["prop_group"],
                                   "member_steps_per_s": nv * steps / el,
                                   "max_abs_docc_diff_vs_default_plan": float(np.max(np.abs(o[:, :, 3] - d64)))}
        print(f"[bench] c64_batch8 on the tuned plan ({label}): {nv * steps / el:.0f} member-steps/s",
              file=sys.stderr, flush=True)
    res["speedup_c64_batch8_vs_plain_c128"] = None  # filled by the caller
    return res


def controller_c5_variant(hub) -> dict:
    """The learned Krylov controller as configured.  Training rows from the
    plain adaptive method (tol 1e-8, default schedule, untimed): the 10-site
    ring (5/5) under 12 seeded U-groups x 8 pulses, 1500 steps of 0.01, and
    the 12-site cluster (6/6) under 4 U-groups x 8 pulses, 1500 steps of
    0.005, from the ground state of H(0) at each U; U ~ U[4, 12], A0 ~
    U[0.2, 1.2], omega ~ U[U/2, 2U], pulses centred at t0 = 1.5 with sigma =
    0.5.  Full-batch Adam on the GPU kernels.  Evaluation on held-out 12-site
    pulses (4 draws of another seed, 1000 steps of 0.005 from the ground state,
    tol 1e-8): steps/s with the learned controller (chunk 16, margin 1 and
    margin 0), the default chunked schedule and the synchronous one, launches per step,
    fallback rate, and bit-identity of the states and logs with the
    synchronous schedule."""
    import numpy as np
    import torch
    from synth import ring, cluster_2d, controller_groups
    from paper_2005_13498_amd import controller as ctl

    tol, chunk, margin = 1e-8, 16, 1
    t0 = time.perf_counter()
    X1, Y1 = ctl.group_runs(hub, ring(10), 5, 5, controller_groups(12, 8, 13500), 1.5, 0.5, 0.01, 1500, tol, chunk)
    X2, Y2 = ctl.group_runs(hub, cluster_2d(3, 4), 6, 6, controller_groups(4, 8, 13501), 1.5, 0.5, 0.005, 1500, tol,
                            chunk)
    X, Y = np.concatenate([X1, X2]), np.concatenate([Y1, Y2])
    t_rows = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, hist = ctl.train(X, Y, steps=1500, lr=3e-3, seed=0, report_every=500)
    t_train = time.perf_counter() - t0
    print(f"[bench] controller: {len(X)} rows in {t_rows:.1f} s, trained in {t_train:.1f} s, loss "
          f"{hist[0][1]:.3f} -> {hist[-1][1]:.4f}", file=sys.stderr, flush=True)
    res = {"train_rows": int(len(X)), "rows_10site": int(len(X1)), "rows_12site": int(len(X2)),
           "rows_seconds_untimed": t_rows, "train_seconds_untimed": t_train,
           "train_loss_first_last": [hist[0][1], hist[-1][1]], "tol": tol, "chunk": chunk, "margin": margin}
    lat = cluster_2d(3, 4)
    n, dt = 1000, 0.005
    opts = hub.make_opts(tol=tol, m_max=30)
    tot = {k: {"seconds": 0.0, "steps": 0, "fallbacks": 0, "launches": 0, "m": 0.0} for k in
           ("learned", "learned_margin0", "default", "synchronous")}
    same = True
    for U, mem in controller_groups(4, 1, 13599):
        B = hub.Basis(lat, U, 6, 6)
        g = torch.empty(B.dim, dtype=torch.complex128, device="cuda:0")
        hub.hub_ground_state(B.handle, 0.0, g, hub.make_opts(tol=1e-10, m_max=60), allow_degenerate=True)
        pulse = (0, mem[0][0], mem[0][1], 1.5, 0.5, 0.0)
        hub.hub_controller_load(B.handle, params)
        ref = None
        for name in ("synchronous", "default", "learned", "learned_margin0"):
            if name.startswith("learned"):
                hub.hub_controller_enable(B.handle, True, chunk, margin if name == "learned" else 0)
            else:
                hub.hub_controller_enable(B.handle, False)
                hub.hub_set_schedule(B.handle, 0 if name == "synchronous" else 32, 0 if name == "synchronous" else 1)
            hub.hub_propagate(B.handle, [pulse], 0.0, dt, 100, opts, g.clone(), want_obs=False)  # warm-up
            v = g.clone()
            hub.hub_controller_read_stats(B.handle)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, obs, log = hub.hub_propagate(B.handle, [pulse], 0.0, dt, n, opts, v)
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            s = hub.hub_controller_read_stats(B.handle)
            T = tot[name]
            T["seconds"] += el
            T["steps"] += n
            T["fallbacks"] += s["fallbacks"]
            T["launches"] += s["lanczos_launches"]
            T["m"] += float(np.sum(log[:, 0, 0]))
            if ref is None:
                ref = (v, obs, log)
            else:
                same &= bool(torch.equal(v, ref[0])) and bool(np.array_equal(obs, ref[1])) and \
                    bool(np.array_equal(log, ref[2]))
        hub.hub_controller_enable(B.handle, False)
        B.close()
    for name, T in tot.items():
        res[name] = {"steps_per_s": T["steps"] / T["seconds"], "mean_krylov_m": T["m"] / T["steps"]}
        if name != "synchronous":
            res[name]["lanczos_launches_per_step"] = T["launches"] / T["steps"]
            res[name]["fallback_rate"] = T["fallbacks"] / T["steps"]
    res["speedup_learned_vs_default"] = res["learned"]["steps_per_s"] / res["default"]["steps_per_s"]
    res["speedup_learned_margin0_vs_default"] = res["learned_margin0"]["steps_per_s"] / res["default"]["steps_per_s"]
    res["speedup_learned_vs_synchronous"] = res["learned"]["steps_per_s"] / res["synchronous"]["steps_per_s"]
    res["bit_identical_to_synchronous"] = same
    print(f"[bench] controller, margin 0: {res['learned_margin0']['steps_per_s']:.0f} steps/s, "
          f"{res['learned_margin0']['lanczos_launches_per_step']:.2f} launches per step, fallback rate "
          f"{res['learned_margin0']['fallback_rate']:.3f}", file=sys.stderr, flush=True)
    print(f"[bench] controller (12 sites, held out): learned {res['learned']['steps_per_s']:.0f}, default "
          f"{res['default']['steps_per_s']:.0f}, synchronous {res['synchronous']['steps_per_s']:.0f} steps/s; "
          f"fallback rate {res['learned']['fallback_rate']:.3f}; bit-identical {same}", file=sys.stderr, flush=True)
    return res


def synchronous_variant(hub, B, w, v_start, t_start: float, steps: int, v_plain, obs_plain, plain_steps_per_s):
    """The same timed workload with the synchronous schedule (one host round
    trip per step) instead of the default chunked one; both must give the
    same bits."""
    import numpy as np
    import torch

    opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
    hub.hub_set_schedule(B.handle, 0, 0)
    v = v_start.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, obs, log = hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, steps, opts, v)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hub.hub_set_schedule(B.handle, 32, 1)
    same = bool(torch.equal(v, v_plain)) and bool(np.array_equal(obs, obs_plain))
    print(f"[bench] synchronous schedule: {steps / el:.0f} steps/s, bit-identical {same}", file=sys.stderr, flush=True)
    return {"steps_per_s": steps / el, "ms_per_step": el / steps * 1e3,
            "default_speedup_over_synchronous": plain_steps_per_s / (steps / el),
            "bit_identical_to_default": same}


def cfet4_variant(hub, B, w, v_start, t_start: float, steps: int, v_plain, plain_seconds: float):
    """Accuracy per cost of the fourth-order commutator-free scheme at 12
    sites: over the timed window of the midpoint run (steps x dt), CFET4 with
    a 4x larger step (two Krylov solves each) is timed and both end states
    are compared with a CFET4 reference at the midpoint run's step (untimed)."""
    import numpy as np
    import torch

    T = steps * w.dt
    opts = hub.make_opts(tol=w.tol, m_max=w.m_max, scheme=1)
    ref = v_start.clone()
    hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, steps, opts, ref, want_obs=False)
    n4 = steps // 4
    v = v_start.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, obs, log = hub.hub_propagate(B.handle, [w.pulse], t_start, 4 * w.dt, n4, opts, v)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nr = float(torch.linalg.vector_norm(ref))
    err4 = float(torch.linalg.vector_norm(v - ref)) / nr
    err2 = float(torch.linalg.vector_norm(v_plain - ref)) / nr
    print(f"[bench] cfet4 dt={4 * w.dt}: {el:.3f} s (midpoint {plain_seconds:.3f} s), |dpsi| {err4:.2e} vs "
          f"midpoint {err2:.2e}", file=sys.stderr, flush=True)
    return {"window": T, "cfet4_dt": 4 * w.dt, "cfet4_steps": n4, "cfet4_seconds": el,
            "midpoint_dt": w.dt, "midpoint_seconds": plain_seconds,
            "cfet4_rel_error_vs_fine_cfet4": err4, "midpoint_rel_error_vs_fine_cfet4": err2,
            "time_ratio_midpoint_over_cfet4": plain_seconds / el,
            "mean_krylov_m_per_solve": float(np.mean(log[:, 0, 0]))}


def large_tile_variant(hub, steps: int = 4, sizes=(14, 16)) -> dict:
    """HBM-resident tiles: the 14-site ring (7/7, 188 MB per complex128 vector)
    and the 16-site ring (8/8, 2.65 GB; down hops gathered from the row in
    global memory).  Per size: the plain H*v's kernel time and algorithmic
    GB/s (HIP events on 10 launches), midpoint steps/s of a few complex128
    steps from a seeded random state under the ring pulse, and, from two more
    steps with HIP events on every Lanczos launch, the average working
    iteration (at 14 sites the fused two-pass pair) against its algorithmic
    4 N s bytes."""
    import numpy as np
    import torch
    from synth import ring, PulseParams

    out = {}
    for ns in sizes:
        half = ns // 2
        B = hub.Basis(ring(ns), 8.0, half, half)
        g = torch.Generator(device="cuda:0").manual_seed(ns)
        x = torch.randn(B.dim, dtype=torch.complex128, device="cuda:0", generator=g)
        x /= torch.linalg.vector_norm(x)
        y = torch.empty_like(x)
        hub.hub_apply_H(B.handle, [0.3], x, y)
        hub.hub_profile_enable(B.handle, 1)
        hub.hub_profile_read(B.handle)
        for _ in range(10):
            hub.hub_apply_H(B.handle, [0.3], x, y)
        n, ms, bpl = hub.hub_profile_read(B.handle)
        hub.hub_profile_enable(B.handle, 0)
        del y
        us = ms / max(n, 1) * 1e3
        p = PulseParams(0, 0.5, 8.0, 0.05, 0.3)
        opts = hub.make_opts(tol=1e-10, m_max=20)
        # untimed steps on a copy for ~0.3 s first: a process's first long
        # propagation runs slower than later ones over the same steps
        xw = x.clone()
        tw = time.perf_counter()
        while True:
            hub.hub_propagate(B.handle, [p], 0.0, 0.01, 1, opts, xw, want_obs=False)
            torch.cuda.synchronize()
            if time.perf_counter() - tw > 0.3:
                break
        del xw
        hub.hub_propagate(B.handle, [p], 0.0, 0.01, 1, opts, x, want_obs=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, obs, log = hub.hub_propagate(B.handle, [p], 0.01, 0.01, steps, opts, x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"ring{ns}"] = {"dim": int(B.dim), "hv_us": us, "hv_bytes": bpl, "hv_gbps": bpl / (us * 1e-6) / 1e9,
                            "hv_frac_of_8TBs": bpl / (us * 1e-6) / 8e12, "steps": steps,
                            "midpoint_steps_per_s": steps / el, "mean_krylov_m": float(np.mean(log[:, 0, 0]))}
        hub.hub_profile_enable(B.handle, 1)
        hub.hub_profile_read(B.handle)
        hub.hub_propagate(B.handle, [p], 0.01 * (steps + 1), 0.01, 2, opts, x, want_obs=False)
        nl, lms, lbpl = hub.hub_profile_read(B.handle)
        hub.hub_profile_enable(B.handle, 0)
        if nl:
            lus = lms / nl * 1e3
            out[f"ring{ns}"].update({"lanczos_launches": nl, "lanczos_us": lus, "lanczos_bytes": lbpl,
                                     "lanczos_gbps": lbpl / (lus * 1e-6) / 1e9,
                                     "lanczos_frac_of_8TBs": lbpl / (lus * 1e-6) / 8e12})
        print(f"[bench] ring{ns}: H*v {us:.0f} us = {bpl / (us * 1e-6) / 1e9:.0f} GB/s, "
              f"{steps / el:.1f} steps/s" + (f"; Lanczos iteration {lms / nl * 1e3:.0f} us = "
                                            f"{lbpl / (lms / nl * 1e-3) / 1e9:.0f} GB/s" if nl else ""),
              file=sys.stderr, flush=True)
        B.close()
        del x
        torch.cuda.empty_cache()
    return out


def ring8_variant(hub) -> dict:
    """The latency case: 8-site ring (U = 8, 4/4, dim 4900) from its ground
    state, 200 steps of 0.01 under the ring pulse, tol 1e-12, complex128
    (a 157 KB apply).  Steps/s on the resident stepper (one launch, the
    default here) and on the launch path with the default and the
    synchronous schedule; then 64 pulses of the same sweep in one call
    (member-steps/s) on both paths."""
    import numpy as np
    import torch
    from synth import PulseParams, workloads

    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn)
    g = torch.empty(B.dim, dtype=torch.complex128, device="cuda:0")
    hub.hub_ground_state(B.handle, hub.hub_pulse_A(w.pulse, 0.0), g, hub.make_opts(tol=1e-13, m_max=100))
    opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
    res = {"dim": int(B.dim), "steps": w.n_steps}

    def timed(pulses, x0, path, chunk=None):
        hub.hub_set_propagate_path(B.handle, path)
        if chunk is not None:
            hub.hub_set_schedule(B.handle, chunk, 0)
        try:
            hub.hub_propagate(B.handle, pulses, 0.0, w.dt, w.n_steps, opts, x0.clone())  # warm-up
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, w.dt, w.n_steps, opts, x)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            hub.hub_set_schedule(B.handle, 32, 1)
            hub.hub_set_propagate_path(B.handle, -1)
        return el, x, obs, log

    el, x_res, obs_res, log = timed([w.pulse], g, 1)
    res["resident"] = {"steps_per_s": w.n_steps / el, "mean_krylov_m": float(np.mean(log[:, 0, 0])),
                       "kernels": "one launch for all steps (one workgroup, tile in LDS)"}
    for name, chunk in (("launches_default", None), ("launches_synchronous", 0)):
        el, x, obs, log = timed([w.pulse], g, 0, chunk)
        res[name] = {"steps_per_s": w.n_steps / el, "mean_krylov_m": float(np.mean(log[:, 0, 0]))}
    res["resident_vs_launches_max_abs_psi_diff"] = float(torch.max(torch.abs(x_res - x)).item())
    res["resident_vs_launches_max_abs_obs_diff"] = float(np.max(np.abs(obs_res[:, :, 1:] - obs[:, :, 1:])))
    res["speedup_resident_vs_launches_default"] = (res["resident"]["steps_per_s"] /
                                                   res["launches_default"]["steps_per_s"])
    # a sweep of 64 amplitudes in one call
    nb = 64
    pulses = [PulseParams(0, 0.1 + 0.8 * k / (nb - 1), w.pulse.omega, w.pulse.t0, w.pulse.sigma) for k in range(nb)]
    xb = g.repeat(nb).contiguous()
    sweep = {"members": nb}
    for name, path in (("resident", 1), ("launches", 0)):
        el, x, obs, log = timed(pulses, xb, path)
        sweep[name] = {"member_steps_per_s": nb * w.n_steps / el, "seconds": el}
    sweep["speedup_resident_vs_launches"] = (sweep["resident"]["member_steps_per_s"] /
                                             sweep["launches"]["member_steps_per_s"])
    res["sweep64"] = sweep
    print(f"[bench] ring8: resident {res['resident']['steps_per_s']:.0f} steps/s, launches "
          f"{res['launches_default']['steps_per_s']:.0f} (synchronous {res['launches_synchronous']['steps_per_s']:.0f});"
          f" 64-pulse sweep {sweep['resident']['member_steps_per_s']:.0f} vs "
          f"{sweep['launches']['member_steps_per_s']:.0f} member-steps/s", file=sys.stderr, flush=True)
    B.close()
    return res


def copy_bandwidth() -> dict:
    """Measured device copy bandwidth (torch copy of 1 GiB, far beyond the
    Infinity Cache): the practical ceiling the kernels are also compared with."""
    import torch

    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    gbps = 2 * nbytes / (ms * 1e-3) / 1e9
    print(f"[bench] copy: {gbps:.0f} GB/s", file=sys.stderr, flush=True)
    return {"bytes_read_plus_written": 2 * nbytes, "ms": ms, "gbps": gbps}


def hv_variants(hub, B, copy_gbps: float, reps: int = 100) -> dict:
    """Plain H*v at 12 sites (A = 0.5 fixed, seeded complex normal x): c128 and
    c64, one vector and blocks of 8.  Per variant the kernel time per apply
    (HIP events on every launch) and the algorithmic GB/s (2 B N s) with the
    same buffers every time (working set in the Infinity Cache) and rotating
    over distinct buffers totalling more than 2 x 256 MB (HBM-served)."""
    import torch

    out = {}
    N = B.dim
    for name, dtype, nv in (("c128x1", torch.complex128, 1), ("c64x1", torch.complex64, 1),
                            ("c64x8", torch.complex64, 8), ("c128x8", torch.complex128, 8)):
        es = 16 if dtype == torch.complex128 else 8
        pair = 2 * nv * N * es
        npairs = max(2, -(-(600 << 20) // pair))  # distinct x/y pairs above 600 MiB
        g = torch.Generator(device="cuda:0").manual_seed(1)
        xs = [torch.randn(nv * N, dtype=dtype, device="cuda:0", generator=g) for _ in range(npairs)]
        ys = [torch.empty_like(xs[0]) for _ in range(npairs)]
        A = [0.5] * nv
        res = {"bytes_per_apply": pair, "buffers_rotated": npairs,
               "kernels": plan_label(hub, B, hub.HUB_C128 if dtype == torch.complex128 else hub.HUB_C64, nv, False)}
        for mode in ("in_cache", "hbm_rotating"):
            for r in range(10):  # untimed: same access pattern as the timed loop
                k = 0 if mode == "in_cache" else r % npairs
                hub.hub_apply_H(B.handle, A, xs[k], ys[k])
            hub.hub_profile_enable(B.handle, 1)
            hub.hub_profile_read(B.handle)
            for r in range(reps):
                k = 0 if mode == "in_cache" else r % npairs
                hub.hub_apply_H(B.handle, A, xs[k], ys[k])
            n, ms, bpl = hub.hub_profile_read(B.handle)
            hub.hub_profile_enable(B.handle, 0)
            # hub_profile counts one launch per vector group: per apply = n / reps groups
            us = ms / reps * 1e3
            gbps = pair / (us * 1e-6) / 1e9
            res[mode] = {"us_per_apply": us, "gbps": gbps, "frac_of_8TBs": gbps / 8000.0,
                         "frac_of_measured_copy": gbps / copy_gbps, "timed_kernel_launches": n}
        out[name] = res
        print(f"[bench] H*v {name}: {res['in_cache']['us_per_apply']:.1f} us in cache "
              f"({res['in_cache']['gbps']:.0f} GB/s), {res['hbm_rotating']['us_per_apply']:.1f} us rotating "
              f"({res['hbm_rotating']['gbps']:.0f} GB/s)", file=sys.stderr, flush=True)
        del xs, ys
        torch.cuda.empty_cache()
    return out


def greens_variant(hub) -> dict:
    """Batched nonequilibrium Green's functions: the 10-site ring (U = 8, 5/5,
    dim 63,504) from its ground state under the ring pulse; 64 members (c and
    c^dag of both spins at sites 0, 3, 6, 9 from t' = 0.5, 1.0, 1.5, 2.0) in
    the four N -/+ 1 sectors (dim 52,920 each), 400 relative steps of 0.01
    each.  complex64 and complex128 runs (Krylov tol 1e-8) on both member
    steppers (persistent one-launch, per-sector batches): member-steps/s, the
    complex64 overlaps' largest deviation from complex128 and the largest
    difference between the steppers."""
    import numpy as np
    import torch
    from synth import workloads

    w = workloads()["ring10_greens"]
    B = hub.Basis(w.lattice, w.U, 5, 5)
    T = [hub.Basis(w.lattice, w.U, *sec) for sec in ((4, 5), (6, 5), (5, 4), (5, 6))]
    g = torch.empty(B.dim, dtype=torch.complex128, device="cuda:0")
    hub.hub_ground_state(B.handle, hub.hub_pulse_A(w.pulse, 0.0), g, hub.make_opts(tol=1e-12, m_max=100))
    members = [(site, spin, dagger, int(round(tp / w.dt)))
               for spin, dagger in ((0, 1), (1, 1), (0, 0), (1, 0))
               for site in w.extra["sites"] for tp in w.extra["t_primes"]]
    n_rel = 400
    opts = hub.make_opts(tol=1e-8, m_max=w.m_max)
    res = {"members": len(members), "relative_steps": n_rel, "member_dim": int(T[0].dim)}
    outs = {}
    for path, pname in ((1, "persistent_members"), (0, "per_sector")):
        hub.hub_set_greens_path(B.handle, path)
        r = res[pname] = {}
        for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
            psi = g.to(dtype).clone()
            hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, 8, opts, members[:4],
                                psi.clone())  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, n_rel, opts, members, psi)
            el = time.perf_counter() - t0
            outs[(pname, name)] = o
            r[name] = {"seconds": el, "member_steps_per_s": len(members) * n_rel / el}
        r["max_abs_overlap_err_c64_vs_c128"] = float(np.max(np.abs(outs[(pname, "c64")] - outs[(pname, "c128")])))
        print(f"[bench] greens ({pname}): c64 {r['c64']['member_steps_per_s']:.0f} member-steps/s, c128 "
              f"{r['c128']['member_steps_per_s']:.0f}; |dG| {r['max_abs_overlap_err_c64_vs_c128']:.1e}",
              file=sys.stderr, flush=True)
    # the per-sector batches again on the committed tuned plans of the target sectors
    from paper_2005_13498_amd import tuning
    tab = tuning.load().get(tuning.device_name(), {})
    if all(tuning.key(t, p) in tab for t in T for p in (hub.HUB_C64, hub.HUB_C128)):
        hub.hub_set_greens_path(B.handle, 0)
        r = res["per_sector_tuned"] = {}
        for name, dtype, prec in (("c64", torch.complex64, hub.HUB_C64), ("c128", torch.complex128, hub.HUB_C128)):
            for t in T:
                hub.hub_set_tuning(t.handle, prec, tab[tuning.key(t, prec)])
            r[name + "_kernels_per_sector"] = plan_label(hub, T[0], prec, len(members) // len(T), True)
            psi = g.to(dtype).clone()
            hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, 8, opts, members[:4], psi.clone())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, n_rel, opts, members, psi)
            el = time.perf_counter() - t0
            r[name] = {"seconds": el, "member_steps_per_s": len(members) * n_rel / el,
                       "max_abs_diff_vs_default_plan": float(np.max(np.abs(o - outs[("per_sector", name)])))}
            for t in T:
                hub.hub_set_tuning(t.handle, prec, None)
        print(f"[bench] greens (per_sector, tuned plans): c64 {r['c64']['member_steps_per_s']:.0f} member-steps/s, "
              f"c128 {r['c128']['member_steps_per_s']:.0f}", file=sys.stderr, flush=True)
    hub.hub_set_greens_path(B.handle, -1)
    res["max_abs_overlap_diff_between_steppers_c128"] = float(
        np.max(np.abs(outs[("persistent_members", "c128")] - outs[("per_sector", "c128")])))
    for t in T:
        t.close()
    B.close()
    return res


def greens_scaling_variant(hub, paths=((1, "persistent_members"), (0, "per_sector"))) -> dict:
    """Member count against stepper: the 10-site ring's Green's-function
    members (c and c^dag of both spins at all 10 sites, t' on a grid from
    0.1) at 256 and 1024 members, 50 relative steps of 0.01, complex64, on
    the persistent member stepper and on the per-sector batches."""
    import numpy as np
    import torch
    from synth import workloads

    w = workloads()["ring10_greens"]
    B = hub.Basis(w.lattice, w.U, 5, 5)
    T = [hub.Basis(w.lattice, w.U, *sec) for sec in ((4, 5), (6, 5), (5, 4), (5, 6))]
    g = torch.empty(B.dim, dtype=torch.complex64, device="cuda:0")
    g.copy_(torch.from_numpy(np.random.default_rng(5).normal(size=B.dim) + 0j).to("cuda:0"))
    g /= torch.linalg.vector_norm(g)
    opts = hub.make_opts(tol=1e-8, m_max=w.m_max)
    n_rel = 50
    res = {"relative_steps": n_rel, "member_dim": int(T[0].dim), "dtype": "c64"}
    for n_tp in (8, 32):
        members = [(site, spin, dagger, 10 * (k + 1))
                   for spin, dagger in ((0, 1), (1, 1), (0, 0), (1, 0)) for site in range(10) for k in range(n_tp)]
        members = members[:(256 if n_tp == 8 else 1024)]
        r = res[f"members_{len(members)}"] = {}
        for path, pname in paths:
            hub.hub_set_greens_path(B.handle, path)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, n_rel, opts, members, g.clone())
            el = time.perf_counter() - t0
            r[pname] = {"seconds": el, "member_steps_per_s": len(members) * n_rel / el}
            print(f"[bench] greens {len(members)} members ({pname}): {len(members) * n_rel / el:.0f} member-steps/s",
                  file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    hub.hub_set_greens_path(B.handle, -1)
    for t in T:
        t.close()
    B.close()
    return res


def ring14_block_variant(hub, steps: int = 40) -> dict:
    """14-site ring (7/7, dim 11,778,624; vectors far beyond the Infinity
    Cache): a complex64 block of 8 pulse amplitudes (A0 = 0.1 .. 0.8) in one
    hub_propagate call against complex128 single-vector calls, from a seeded
    random state: member-steps/s of both and the complex64 block's largest
    deviation in d(t) and E(t)/N_s from complex128 (same member)."""
    import numpy as np
    import torch
    from synth import workloads, PulseParams

    w = workloads()["ring14_block"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn)
    pulses = [PulseParams(0, a, w.pulse.omega, w.pulse.t0, w.pulse.sigma) for a in w.extra["A0_batch"]]
    g = torch.Generator(device="cuda:0").manual_seed(14)
    x0 = torch.randn(B.dim, dtype=torch.complex128, device="cuda:0", generator=g)
    x0 /= torch.linalg.vector_norm(x0)
    opts = hub.make_opts(tol=1e-8, m_max=w.m_max)
    res = {"dim": int(B.dim), "members": len(pulses), "steps": steps}
    xb = x0.to(torch.complex64).repeat(len(pulses)).contiguous()
    hub.hub_propagate(B.handle, pulses, 0.0, w.dt, 1, opts, xb.clone(), want_obs=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, obs64, log64 = hub.hub_propagate(B.handle, pulses, 0.0, w.dt, steps, opts, xb)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    del xb
    torch.cuda.empty_cache()
    obs128 = []
    el128 = 0.0
    for p in pulses:
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, o, lg = hub.hub_propagate(B.handle, [p], 0.0, w.dt, steps, opts, x)
        torch.cuda.synchronize()
        el128 += time.perf_counter() - t0
        obs128.append(o[:, 0, :])
        del x
    obs128 = np.stack(obs128, axis=1)
    res["c64_8members"] = {"kernels": plan_label(hub, B, hub.HUB_C64, len(pulses), True),
                         "seconds": el64, "member_steps_per_s": len(pulses) * steps / el64,
                         "mean_krylov_m": float(np.mean(log64[:, :, 0]))}
    res["c128_single"] = {"seconds": el128, "member_steps_per_s": len(pulses) * steps / el128}
    tr = tuned_run(hub, B, hub.HUB_C64, pulses, 0.0, w.dt, steps, opts,
                   x0.to(torch.complex64).repeat(len(pulses)).contiguous())
    if tr is not None:
        ent, label, el, o = tr
        res["c64_8members_tuned"] = {"kernels": label, "prop_group": ent["prop_group"], "seconds": el,
                                     "member_steps_per_s": len(pulses) * steps / el,
                                     "max_abs_docc_diff_vs_default_plan": float(np.max(np.abs(o[:, :, 3] - obs64[:, :, 3])))}
        print(f"[bench] ring14 c64 8 members on the tuned plan ({label}): "
              f"{len(pulses) * steps / el:.1f} member-steps/s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    res["max_abs_docc_err"] = float(np.max(np.abs(obs64[:, :, 3] - obs128[:, :, 3])))
    res["max_abs_energy_per_site_err"] = float(np.max(np.abs(obs64[:, :, 2] - obs128[:, :, 2])))
    print(f"[bench] ring14: c64 8 members {res['c64_8members']['member_steps_per_s']:.1f} member-steps/s, c128 "
          f"{res['c128_single']['member_steps_per_s']:.1f}; |dd| {res['max_abs_docc_err']:.1e}",
          file=sys.stderr, flush=True)
    B.close()
    del x0
    torch.cuda.empty_cache()
    return res


def run_cpu_allcores(seconds: float) -> dict:
    """All-cores oracle figure for the batched configuration: one single-threaded
    oracle process per member of the 8-pulse batch (at most one per host CPU),
    run side by side; member-steps/s summed."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    n = max(1, min(8, os.cpu_count() or 1))
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-seconds",
                               str(seconds), "--cpu-member", str(k)], env=env, stdout=subprocess.PIPE,
                              stderr=subprocess.PIPE, text=True) for k in range(n)]
    out = []
    for pr in procs:
        so, se = pr.communicate(timeout=900)
        if pr.returncode != 0:
            return {"error": se[-500:]}
        out.append(json.loads(so.strip().splitlines()[-1]))
    total = sum(o["steps_per_s"] for o in out)
    return {"processes": n, "member_steps_per_s": total, "unit": "member midpoint steps/s",
            "sample": f"{n} oracle processes side by side, one batch member each, ~{seconds:.0f} s of steps each"}


def run_cpu_baseline_child(seconds: float) -> dict:
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                        "--cpu-seconds", str(seconds)], env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    # the first long propagation of a process runs ~13% slower than later
    # ones over the same steps; the default warmup covers it
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-member", type=int, default=-1, help=argparse.SUPPRESS)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain copy of known size (counter scaling)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"))
    ap.add_argument("--summarize-stats", nargs=2, metavar=("TRACE_DIR", "OUT"))
    ap.add_argument("--counters-case", choices=tuple(COUNTER_CASES), default="cluster3x4",
                    help="workload whose fused Lanczos pair --summarize-counters reads")
    ap.add_argument("--command", default="", help="profiling command recorded in a summary")
    ap.add_argument("--note", default="", help="comment lines (separated by |) recorded in a summary")
    ap.add_argument("--variant", choices=("greens_ring10", "greens_scaling", "greens_persistent", "ring14_block",
                                          "ring8", "hv12", "controller", "ring14"),
                    help="run only this variant and print its result (for profiling it alone)")
    args = ap.parse_args()

    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_seconds, args.cpu_member)))
        return 0
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, command=args.command, case=args.counters_case)
        return 0
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, command=args.command, note=args.note)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(batches would shard across GPUs with no communication).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2005_13498_amd as hub
    from synth import workloads

    if args.variant:
        torch.cuda.set_device(0)
        if args.variant == "hv12":
            w = workloads()["cluster3x4"]
            B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
            print(json.dumps({"hv_12site": hv_variants(hub, B, copy_bandwidth()["gbps"])}), flush=True)
            B.close()
            return 0
        run = {"greens_ring10": greens_variant, "greens_scaling": greens_scaling_variant,
               "greens_persistent": lambda h: greens_scaling_variant(h, ((1, "persistent_members"),)),
               "ring14_block": ring14_block_variant, "ring8": ring8_variant,
               "controller": controller_c5_variant, "ring14": lambda h: large_tile_variant(h, sizes=(14,))}
        print(json.dumps({args.variant: run[args.variant](hub)}), flush=True)
        if args.copy_calibration:
            copy_calibration()
        return 0

    w = workloads()["cluster3x4"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    print(f"[bench] setup {w.name} dim={len(w.lattice.bonds)} bonds", file=sys.stderr, flush=True)
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    v = torch.empty(B.dim, dtype=torch.complex128, device=dev)
    A0 = hub.hub_pulse_A(w.pulse, 0.0)
    st, e0, gap = hub.hub_ground_state(B.handle, A0, v, hub.make_opts(tol=1e-12, m_max=100))
    print(f"[bench] ground state E0={e0:.12f} gap={gap:.4f}", file=sys.stderr, flush=True)
    v0 = v.clone()
    opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
    stream = torch.cuda.current_stream()

    # The timed window is centred on the pulse whatever K is: the ground state
    # of H(0) is first advanced (untimed, part of the setup like the ground
    # state itself) to t_s = max(0, t0 - K dt / 2), the nearest step.  W
    # warm-up steps then run from t_s on a copy, and the K timed steps from t_s.
    n_pre = max(0, int(round((w.pulse.t0 - 0.5 * args.steps * w.dt) / w.dt)))
    t_start = n_pre * w.dt
    if n_pre > 0:
        hub.hub_propagate(B.handle, [w.pulse], 0.0, w.dt, n_pre, opts, v, want_obs=False, want_log=False,
                          stream=stream)
    if args.warmup > 0:
        vw = v.clone()
        hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, args.warmup, opts, vw, stream=stream)
        del vw
    torch.cuda.synchronize()

    v_start = v.clone()
    # events on every p-th fused iteration, at least ~20 of them in the window
    # (a step has m - 1 ~ 5 fused iterations that do work in the pulse)
    period = max(1, min(PROFILE_PERIOD, (5 * args.steps) // 20))
    # timed region: exactly K midpoint steps
    hub.hub_profile_enable(B.handle, period)
    hub.hub_profile_read(B.handle)  # reset counters
    hub.hub_controller_read_stats(B.handle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, obs, log = hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, args.steps, opts, v, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kernel_ms, bytes_per = hub.hub_profile_read(B.handle)
    hub.hub_profile_enable(B.handle, False)
    sched = hub.hub_controller_read_stats(B.handle)
    elapsed = t1 - t0
    steps_per_s = args.steps / elapsed
    avg_us = kernel_ms / max(launches, 1) * 1e3
    achieved = bytes_per / (avg_us * 1e-6) / 1e9 if launches else 0.0
    mean_m = float(np.mean(log[:, 0, 0])) if log is not None else None
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s; H*v launches {launches}, avg {avg_us:.2f} us, "
          f"{achieved:.0f} GB/s; mean m {mean_m}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "midpoint steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cluster3x4 12-site periodic, U=8, 6/6 (dim 853776), FP64 single vector, "
                               "dt=0.005, tol=1e-10, window of K steps centred on the pulse (ground state of H(0) advanced untimed)",
                   "A0": w.pulse.A0, "omega": w.pulse.omega, "t0": w.pulse.t0, "sigma": w.pulse.sigma,
                   "t_window": [t_start, t_start + args.steps * w.dt], "untimed_steps_before_window": n_pre,
                   "max_abs_A_in_window": max(abs(hub.hub_pulse_A(w.pulse, t_start + (k + 0.5) * w.dt))
                                              for k in range(args.steps)) if args.steps else 0.0,
                   "mean_krylov_m": mean_m,
                   "schedule": {"kind": "chunked, 32 steps, margin 1", "chunks": sched["chunks"],
                                "fallback_steps": sched["fallbacks"],
                                "lanczos_launches_per_step": sched["lanczos_launches"] / max(1, sched["steps"])}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "fused Lanczos iteration, complex128: k_apply row pass (forms u_j, diagonal, down hops) "
                               "+ k_colpass (up hops, Lanczos epilogue, Krylov decision)",
                     "bytes_per_launch": bytes_per, "avg_launch_us": avg_us,
                     "timed_launches": launches, "event_sampling": f"every {period}th fused iteration",
                     "trace": trace_figure(bytes_per),
                     "kernels": "sum of both kernel times; bytes = 4 N s (read w_{j-1}, u_{j-1}; write u_j, y)"},
    }
    if args.copy_calibration:
        copy_calibration()
    if not args.no_variants:
        var = {}
        var["copy"] = copy_bandwidth()
        var["ring8"] = ring8_variant(hub)
        var["hv_12site"] = hv_variants(hub, B, var["copy"]["gbps"])
        var.update(batched_variants(hub, B, v_start, t_start, w, args.steps))
        var["synchronous_schedule"] = synchronous_variant(hub, B, w, v_start, t_start, args.steps, v, obs,
                                                          steps_per_s)
        var["controller"] = controller_c5_variant(hub)
        var["cfet4"] = cfet4_variant(hub, B, w, v_start, t_start, args.steps, v, elapsed)
        var["large_tiles"] = large_tile_variant(hub)
        var["greens_ring10"] = greens_variant(hub)
        var["ring14_block"] = ring14_block_variant(hub)
        var["speedup_c64_batch8_vs_plain_c128"] = var["c64_batch8"]["member_steps_per_s"] / steps_per_s
        out["variants"] = var
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline_child(args.cpu_seconds)
        out["cpu_baseline"]["allcores_batch8"] = run_cpu_allcores(10.0)
    B.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
