"""Benchmark: FP64 trajectory-steps/s with tangents on one MI355X.

Workload (one "step" of this benchmark = one whole pass of the hot path):
Henon-Heiles 1024x1024 surface-of-section grids at E = 0.125 and E = 1/6
(x = 0, y in [-0.4, 0.7], p_y in [-0.45, 0.45], p_x >= 0 from the energy,
inaccessible points masked: 850,874 + 992,552 orbits), FP64 Yoshida-4 with
dt = 0.01 to T = 1e4 (1e6 steps), with in one pass: SALI and GALI_2 from two
seeded unit deviation vectors, the 4-exponent Lyapunov spectrum (modified
Gram-Schmidt every 10 steps), the LD M-function (p = 1/2) and the energy
error.  Each pass builds the grids on the GPU, compacts the masks and
integrates both energies as one ensemble.

value = orbit-steps per second over the timed passes (inputs resident in
HBM).  roofline: the integration kernel's algorithmic FP64 flops per launch
(flop model in the design doc) divided by its mean launch duration measured with
HIP events on the stream it runs on.  cpu_baseline: the oracle on this
host's cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12  # MI355X FP64 vector peak, FLOP/s (FMA = 2)

# Sources of the benchmarked integration kernel: the HBM traffic recorded in
# profiles/ applies only while their hash is the one recorded beside it.
KERNEL_SOURCES = ["paper_2507_00622_amd/csrc/lane_kernel.h",
                  "paper_2507_00622_amd/csrc/systems.h",
                  "paper_2507_00622_amd/csrc/device_math.h",
                  "paper_2507_00622_amd/csrc/chx_internal.h",
                  "paper_2507_00622_amd/csrc/lane_hh.hip"]
TRAFFIC_FILE = "profiles/lane_kernel_hh6_traffic.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy), or None when the kernel changed since."""
    try:
        txt = open(os.path.join(ROOT, TRAFFIC_FILE)).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and line.strip().startswith(("kernel-source-sha256", "traffic-bytes-per-launch")):
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel-source-sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic-bytes-per-launch"])
    except (KeyError, ValueError):
        return None


def flops_per_step(N, m_s, n_l, ld, energy, sali, K, system="hh"):
    """Algorithmic FP64 flops of one orbit-step of the lane-per-orbit path
    for Henon-Heiles (FMA = 2, add/mul = 1; sqrt, division, log and
    exponent bookkeeping = 0): the minimal operation count of the step as
    the method is formulated here -- 3 drifts and 3 force evaluations; 4
    state kicks (the LD needs p at every step endpoint) but 3 kicks of the
    deviation vectors (kicks commute, so K(d3) K(d0) is one kick), each
    with the step-scaled Hessian; checkpoint work divided by K."""
    assert system == "hh" and N == 2
    M = m_s + n_l
    D = 2 * N
    force = 2 + 4            # F_x = x(1+2y): 1 FMA; F_y = y - y^2 + x^2: 2 FMA
    hess_scaled = 2 + 1 + 2  # h(1+2y), 2h x, h(1-2y)
    state = 3 * 2 * N + 4 * 2 * N + 3 * force  # drifts, kicks, forces
    vec = 3 * (N * N * 2) + 3 * (N * 2)  # 3 kicks (2x2 mat-vec FMA) + 3 drifts
    per = state + 3 * hess_scaled + M * vec
    if ld:
        per += (2 * N - 1) + 1 + 2  # sum of 2N roots, g_prev + g, FMA into LD
    ck = 0
    norm = 2 * D - 1 + D + 1  # |w|^2, rescale, growth product
    ck += m_s * norm
    if sali:
        ck += 2 * (D + 2 * D - 1)  # |w1 +- w2|^2
    for j in range(n_l):
        ck += j * ((2 * D - 1) + 2 * D) + norm  # projections + normalisation
    if energy:
        ck += 14  # H (kinetic 2 FMA, potential 5 ops) and |H - H0|
    return per + ck / K


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=1024, help="grid side per energy")
    ap.add_argument("--T", type=float, default=1e4)
    ap.add_argument("--steps-per-launch", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="orbits in the oracle sample (strided over the workload)")
    ap.add_argument("--cpu-T", type=float, default=1e4)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this path has no multi-GPU form "
              "(orbits are independent; the sharding design is in DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2507_00622_amd as P
    from paper_2507_00622_amd import chx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes}), flush=True)
        return
    energies = (0.125, 1.0 / 6.0)
    n_side = args.grid
    dt, T, K = 0.01, args.T, 10
    ind = chx.IND_SALI | chx.IND_GALI | chx.IND_LYAP | chx.IND_LD | chx.IND_ENERGY
    opts = dict(dt=dt, T=T, indicators=ind, gali_kmax=2, n_lyap=4, renorm_every=K,
                seed=1002, escape_r2=4.0, block_size=args.block)
    n_steps = int(round(T / dt))
    spl = args.steps_per_launch or 25000
    spl = min(spl, n_steps)
    stream = torch.cuda.current_stream()

    kernel_ms = []

    def one_pass(record):
        xs, ms = [], []
        for E in energies:
            x, m = P.grid_hh_section(E, n_side, n_side, device=dev)
            xs.append(x)
            ms.append(m)
        x0 = torch.cat(xs)
        mask = torch.cat(ms)
        e = P.Ensemble(P.henon_heiles(), x0, mask=mask, steps_per_launch=spl,
                       outputs=("status", "label", "sali_min", "gali", "lyap", "ld",
                                "energy_err"), **opts)
        s = 0
        while s < n_steps:
            nxt = min(s + spl, n_steps)
            if record:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                e.advance(nxt)
                b.record(stream)
                kernel_ms.append((a, b, nxt - s))
            else:
                e.advance(nxt)
            s = nxt
        out = e.results()
        n_active = e.info()[2]
        e.close()
        return out, n_active

    for _ in range(args.warmup):
        one_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_active = 0
    for _ in range(args.steps):
        out, n_active = one_pass(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    orbit_steps = n_active * n_steps * args.steps
    value = orbit_steps / elapsed
    fps = flops_per_step(2, 2, 4, True, True, True, K)
    # dominant kernel: the integration launches (full-length ones)
    full = [(a.elapsed_time(b), n) for a, b, n in kernel_ms if n == spl]
    ms_avg = float(np.mean([t for t, _ in full])) if full else float("nan")
    flops_launch = fps * n_active * spl
    achieved = flops_launch / (ms_avg * 1e-3)
    status = out["status"].cpu().numpy()
    lab = out["label"].cpu().numpy()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, energies, n_side, dt, K)

    line = {
        "metric": "FP64 trajectory-steps/s (with tangents)",
        "value": value,
        "unit": "orbit-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"henon-heiles {n_side}x{n_side} section grids at E=0.125 and "
                        f"E=1/6, dt={dt}, T={T:g}, SALI+GALI_2+4 Lyapunov (MGS/10)"
                        "+LD(p=0.5)+energy in one pass",
            "orbits": int(n_active),
            "steps_per_orbit": n_steps,
            "deviation_vectors": 6,
            "steps_per_launch": spl,
            "chaotic_fraction": float(np.mean(lab[lab >= 0] == 1)),
            "escaped_or_nonfinite": int(np.sum((status == 2) | (status == 3))),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64,
            "traffic": recorded_traffic(),
            "kernel": "chx::lane_kernel<SysHH, 6, false>",
            "flops_per_orbit_step": fps,
            "launch_ms": ms_avg,
            "launches_timed": len(full),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(args, energies, n_side, dt, K):
    """The oracle, as it stands, on this host's cores: a strided sample of the
    workload's orbits (both energies) for T = cpu_T."""
    import numpy as np

    import seeded_inputs as S
    from oracle import oracle as O
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    xs = []
    for E in energies:
        x0, m = O.hh_grid(E, n_side, n_side)
        xs.append(x0[m == 1])
    x = np.concatenate(xs)
    idx = np.linspace(0, len(x) - 1, args.cpu_sample).astype(int)
    xs = x[idx]
    w0 = S.deviation_vectors(1002, len(xs), 2, 4)
    run = O.Run(dt=dt, T=args.cpu_T, indicators=31, gali_kmax=2, n_lyap=4, K=K, escape_r2=4.0)
    t0 = time.perf_counter()
    O.integrate(O.henon_heiles(), xs, run, w0=w0, threads=threads)
    el = time.perf_counter() - t0
    n = len(xs) * int(round(args.cpu_T / dt))
    return {"value": n / el, "unit": "orbit-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(xs)} orbits strided over both grids, T={args.cpu_T:g} "
                      f"({n:.3g} orbit-steps, {el:.1f} s)"}


if __name__ == "__main__":
    main()
