#!/usr/bin/env python3
"""Benchmark of the exponential-midpoint / Krylov time stepper on one MI355X.

Workload (one "step" = one midpoint step: every Lanczos iteration's
matrix-free H*v, the FP64 recurrence and small exponential, the combine, and
the fused observables): 12-site 3x4 periodic cluster, t = 1, U = 8, half
filling 6/6 (dim 853,776), field along x with A0 drawn from the seeded
uniform [0.2, 1.0], omega = 8, sigma = 0.5, t0 = 2.5; dt = 0.005, Krylov
tol 1e-10, m_max 30; single complex128 vector started from the ground state
of H(0).  All inputs synthetic and resident in HBM before timing.

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


def cpu_baseline(seconds: float) -> dict:
    """Oracle timing on the host (run in a single-threaded child process)."""
    import numpy as np
    from synth import workloads, random_state
    from oracle import HubbardOracle, pulse_A, krylov_step_alg6

    w = workloads()["cluster3x4"]
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
    return {"value": steps / el, "unit": "midpoint steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} literal Alg.6 midpoint steps of the 12-site 3x4 workload from the "
                      f"oracle ground state (scipy CSR complex128, tol {w.tol:g}, dt {w.dt}, mean m "
                      f"{float(np.mean(ms)):.2f}, {hv} H*v in {el:.1f} s, 1 thread)"}


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
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    args = ap.parse_args()

    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_seconds)))
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

    w = workloads()["cluster3x4"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    print(f"[bench] setup {w.name} dim={len(w.lattice.bonds)} bonds", file=sys.stderr, flush=True)
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    v = torch.empty(B.dim, dtype=torch.complex128, device=dev)
    A0 = hub.hub_pulse_A(w.pulse, 0.0)
    st, e0, gap = hub.hub_ground_state(B.handle, A0, v, hub.make_opts(tol=1e-12, m_max=100))
    print(f"[bench] ground state E0={e0:.12f} gap={gap:.4f}", file=sys.stderr, flush=True)
    opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
    stream = torch.cuda.current_stream()

    # warmup (untimed)
    t_start = 0.0
    if args.warmup > 0:
        hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, args.warmup, opts, v, stream=stream)
        t_start += args.warmup * w.dt
    torch.cuda.synchronize()

    # timed region: exactly K midpoint steps
    hub.hub_profile_enable(B.handle, True)
    hub.hub_profile_read(B.handle)  # reset counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, obs, log = hub.hub_propagate(B.handle, [w.pulse], t_start, w.dt, args.steps, opts, v, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kernel_ms, bytes_per = hub.hub_profile_read(B.handle)
    hub.hub_profile_enable(B.handle, False)
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
                               "dt=0.005, tol=1e-10, ground-state start",
                   "A0": w.pulse.A0, "omega": w.pulse.omega, "t0": w.pulse.t0, "sigma": w.pulse.sigma,
                   "mean_krylov_m": mean_m, "hv_launches": launches},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_apply (matrix-free H*v, Lanczos epilogue)",
                     "bytes_per_launch": bytes_per, "avg_launch_us": avg_us},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline_child(args.cpu_seconds)
    B.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
