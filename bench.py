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
(model_flops_hh: state, tangent vectors, LD and checkpoint work per
orbit-step, FMA = 2) divided by its mean launch duration measured with
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
PEAK_BF16 = 2.5e15  # MI355X dense BF16 matrix peak, FLOP/s

# The benchmarked integration kernel: the HBM traffic recorded in profiles/
# applies only while the kernel's machine code (its gfx950 instructions and
# kernel descriptor in the built library) hashes to the value recorded
# beside it.
KERNEL_SYMBOL = "_ZN3chx11lane_kernelINS_5SysHHELi6ELb0ELi2EEEvNS_8StepArgsE"
LIBRARY = "paper_2507_00622_amd/libchx.so"
TRAFFIC_FILE = "profiles/lane_kernel_hh6_traffic.md"


def _code_objects(data, arch="gfx950"):
    """The arch's device code objects in the (uncompressed) clang offload
    bundles embedded in a host shared library."""
    import struct
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    out, i = [], data.find(magic)
    while i >= 0:
        p = i + len(magic)
        (num,) = struct.unpack_from("<Q", data, p)
        p += 8
        for _ in range(num):
            off, size, idlen = struct.unpack_from("<QQQ", data, p)
            p += 24
            ident = data[p:p + idlen].decode(errors="replace")
            p += idlen
            if arch in ident and size:
                out.append(data[i + off:i + off + size])
        i = data.find(magic, i + 1)
    return out


def _elf_symbol_bytes(co, names):
    """Bytes of the named symbols (value and size from the ELF64 symbol
    table, located through their sections) of one code object."""
    import struct
    e_shoff, = struct.unpack_from("<Q", co, 0x28)
    e_shentsize, e_shnum = struct.unpack_from("<HH", co, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", co, e_shoff + k * e_shentsize)
            for k in range(e_shnum)]
    found = {}
    for s in secs:
        if s[1] != 2:  # SHT_SYMTAB
            continue
        strtab = secs[s[6]]
        for k in range(s[5] // s[9]):
            name_off, _, _, shndx, value, size = struct.unpack_from("<IBBHQQ", co, s[4] + k * s[9])
            end = co.find(b"\0", strtab[4] + name_off)
            name = co[strtab[4] + name_off:end].decode(errors="replace")
            if name in names and 0 < shndx < len(secs):
                sec = secs[shndx]
                start = sec[4] + value - sec[3]
                found[name] = co[start:start + size]
    return found


def kernel_code_hash(symbol=KERNEL_SYMBOL, lib=LIBRARY):
    """sha256 over a kernel's machine code and its kernel descriptor in the
    built library, or None if it is not there."""
    import hashlib
    try:
        data = open(os.path.join(ROOT, lib), "rb").read()
    except OSError:
        return None
    for co in _code_objects(data):
        b = _elf_symbol_bytes(co, {symbol, symbol + ".kd"})
        if symbol in b and symbol + ".kd" in b:
            return hashlib.sha256(b[symbol] + b[symbol + ".kd"]).hexdigest()
    return None


def recorded_traffic():
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy), or None when the kernel changed since."""
    try:
        txt = open(os.path.join(ROOT, TRAFFIC_FILE)).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and line.strip().startswith(("kernel-code-sha256", "traffic-bytes-per-launch")):
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    h = kernel_code_hash()
    if h is None or vals.get("kernel-code-sha256") != h:
        return None
    try:
        return float(vals["traffic-bytes-per-launch"])
    except (KeyError, ValueError):
        return None


def model_flops_hh(m_s, n_l, ld, sali, K):
    """Algorithmic FP64 flops per orbit-step of Henon-Heiles under Yoshida-4
    by the path's flop model (FMA = 2, add/sub/mul = 1; sqrt, division, log
    = 0): the state 70 (3 force and Hessian evaluations of 10, 4 kicks of 4,
    the Hessian scaled for the 4 kicks 12, 3 drifts of 4), 44 per tangent
    vector (4 kicks of 8, 3 drifts of 4), the LD 6 per step, and per
    checkpoint (divided by K) the renormalised SALI pair 44 and the modified
    Gram-Schmidt of 4 Lyapunov vectors 134.  This is the count of the
    method as stated; the kernel merges commuting kicks and does fewer
    (flops_per_step)."""
    if (m_s, n_l) not in ((2, 0), (2, 4)) or not sali:
        raise ValueError("the flop model covers the SALI pair with 0 or 4 Lyapunov vectors")
    per = 70 + 44 * (m_s + n_l) + (6 if ld else 0)
    return per + (44 + (134 if n_l == 4 else 0)) / K


def model_flops_fput(N, n_l, m_g, K):
    """The same model for an FPU-beta chain of N masses: the state 42N + 19
    (3 force evaluations of 8N + 5, 4 kicks of 2N, the stiffnesses scaled
    for the kicks 4N + 4, 3 drifts of 2N), 22N per tangent vector (4 kicks
    of 4N, 3 drifts of 2N), and per checkpoint (divided by K) the modified
    Gram-Schmidt of the 2N Lyapunov vectors 16N^3 + 4N^2 and the
    renormalisation of the N GALI vectors 6N^2."""
    if n_l not in (0, 2 * N) or m_g not in (0, N, 2):
        raise ValueError("the flop model covers 2N Lyapunov and N (or 2 SALI) vectors")
    per = 42 * N + 19 + 22 * N * (n_l + m_g)
    ck = (16 * N ** 3 + 4 * N ** 2 if n_l else 0) + (6 * N ** 2 if m_g == N else 0) + \
        (12 * N + 8 if m_g == 2 else 0)
    return per + ck / K


def model_flops_quartic(m, sali=True):
    """The path's flop model for the coupled quartic oscillators with 3
    degrees of freedom: the state 147 (3 force and Hessian evaluations of
    27, 4 kicks of 6, the Hessian scaled for the kicks 24, 3 drifts of 6), 90
    per tangent vector, the SALI pair about 7 per step."""
    return 147 + 90 * m + (7 if sali else 0)


def mlp_train_flops_per_row(padded=False):
    """Flops of the gate's products for one row in one training epoch: the
    forward pass 6 -> 256 -> 256 -> 2, the weight gradients of the three
    layers and the activation gradients of the two hidden layers (the input
    needs none).  padded=True counts the products as the matrix cores run
    them, on 16 inputs and 16 logits."""
    i, h, o = (16, 256, 16) if padded else (6, 256, 2)
    layers = i * h + h * h + h * o
    return 2 * layers + 2 * layers + 2 * (o * h + h * h)


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
    return per + checkpoint_flops_hh(N, m_s, n_l, energy, sali) / K


# Non-zero pattern of the DOP853 tableau: entries a_ij (j < i) per stage
# i = 1..12 and the stages with a non-zero weight b_i in the eighth-order
# solution (stages 2..5 have none).
DOP853_ROW_NNZ = (0, 1, 2, 2, 3, 3, 4, 5, 6, 7, 8, 9)
DOP853_B_NNZ = 8


# The double pendulum's field (systems_dp.h), in flops with every add, mul
# and division counted 1 (so an FMA 2), negations and selects free: the
# field from the sines and cosines of the angles 39; the derivative parts of
# its dual-number evaluation along one direction 77 (the value parts are the
# state's); one sincos_cw 69 (the reduction with its two-sums 28, the two
# Taylor polynomials 26, the combinations 15); the energy at a checkpoint 80
# (three cosines at 20 and the quadratic form).
DP_FIELD, DP_JVP, DP_SINCOS, DP_ENERGY = 39, 77, 69, 80


def flops_per_step_dop853(N, m_s, n_l, ld, energy, sali, K, system="hh"):
    """Algorithmic FP64 flops of one orbit-step of the fixed-step DOP853
    lane kernel for Henon-Heiles or the double pendulum (same conventions
    as flops_per_step): per stage the stage input (one FMA per non-zero a_ij
    and component, plus the add to the step's start value), one force
    (state) or step-scaled Hessian and its mat-vec (vectors) -- for the
    double pendulum two sincos and the field (state) or the derivative
    parts of the dual-number evaluation (vectors) -- the h-scaling of the stage
    derivative; the final combination (one FMA per non-zero b_i and
    component, one add); the LD integrand at every stage with a weight;
    checkpoints as for Yoshida-4, divided by K."""
    assert system in ("hh", "dp") and N == 2
    M = m_s + n_l
    D = 2 * N
    sums = 2 * D * sum(DOP853_ROW_NNZ) + D * (len(DOP853_ROW_NNZ) - 1)
    final = 2 * D * DOP853_B_NNZ + D
    if system == "hh":
        force = 2 + 4
        hess_scaled = 2 + 1 + 2
        state = sums + 12 * force + 12 * D + final
        vec = sums + 12 * (hess_scaled + 2 * N * N + N) + final
        e_cost = 14
    else:
        state = sums + 12 * (2 * DP_SINCOS + DP_FIELD + D) + final
        vec = sums + 12 * (DP_JVP + D) + final
        e_cost = DP_ENERGY
    per = state + M * vec
    if ld:
        per += DOP853_B_NNZ * ((2 * N - 1) + 2) + 2
    return per + checkpoint_flops_hh(N, m_s, n_l, energy, sali, e_cost) / K


def flops_per_attempt_dop853(N, m_s, n_l, ld, system="hh"):
    """Algorithmic FP64 flops of one attempted step of the adaptive DOP8(5)
    kernel: the fixed step's work (flops_per_step_dop853 without
    checkpoints) plus the error estimate -- per component of the state and
    the vectors, the fifth-order difference (one FMA per weighted stage),
    the third-order difference (3 FMA), the scale
    atol + rtol max(|y|, |y_new|) (FMA) and two squared ratios (FMA each) --
    and the controller (a handful of operations, counted as 8)."""
    assert system in ("hh", "dp") and N == 2
    D = 2 * N
    comps = D * (1 + m_s + n_l)
    err = comps * (2 * DOP853_B_NNZ + 2 * 3 + 2 + 2 * 2)
    return flops_per_step_dop853(N, m_s, n_l, ld, False, False, 1 << 62, system) + err + 8


def checkpoint_flops_hh(N, m_s, n_l, energy, sali, energy_cost=14):
    """Flops of one checkpoint: renormalisation of the SALI/GALI set, SALI,
    modified Gram-Schmidt of the Lyapunov set, energy (Henon-Heiles: 14)."""
    D = 2 * N
    ck = 0
    norm = 2 * D - 1 + D + 1  # |w|^2, rescale, growth product
    ck += m_s * norm
    if sali:
        ck += 2 * (D + 2 * D - 1)  # |w1 +- w2|^2
    for j in range(n_l):
        ck += j * ((2 * D - 1) + 2 * D) + norm  # projections + normalisation
    if energy:
        ck += energy_cost  # Henon-Heiles: kinetic 2 FMA, potential 5 ops, |H - H0|
    return ck


def flops_per_step_fput(N, m_s, n_l, ld, energy, sali, K):
    """Algorithmic FP64 flops of one orbit-step of an FPU-beta chain of N
    masses between fixed walls (same conventions as flops_per_step): each
    force evaluation takes the N+1 spring elongations (1), forces
    d (k + d (alpha + beta d)) (2 FMA + 1 mul), the net forces (1 per mass)
    and the N+1 stiffnesses k + d (2 alpha + 3 beta d) (2 FMA) of the
    tridiagonal Hessian; a tangent kick scales the three diagonals by the
    kick's step (4 per mass, shared by all vectors) and applies them
    (3 FMA per component)."""
    M = m_s + n_l
    D = 2 * N
    force = 6 * (N + 1) + N + 4 * (N + 1)
    state = 3 * force + 4 * 2 * N + 3 * 2 * N
    prescale = 3 * 4 * N
    vec = 3 * 3 * 2 * N + 3 * 2 * N
    per = state + prescale + M * vec
    if ld:
        per += (2 * N - 1) + 1 + 2
    norm = 2 * D - 1 + D + 1
    ck = m_s * norm
    if sali:
        ck += 2 * (D + 2 * D - 1)
    for j in range(n_l):
        ck += j * ((2 * D - 1) + 2 * D) + norm
    if energy:
        ck += 8 * (N + 1) + 2 * N + 2
    return per + ck / K


def flops_per_step_quartic(N, m_s, ld, energy, sali, K):
    """Algorithmic FP64 flops of one orbit-step of the coupled quartic
    oscillators V = sum q_i^4/4 + eps sum_{i<j} q_i^2 q_j^2 (same
    conventions): force q_i (a q_i^2 + 2 eps S) with S = |q|^2, and the
    step-scaled symmetric Hessian, 3 times per step."""
    D = 2 * N
    force = 2 * N + 1 + 4 * N
    hess = 2 * N + 3 + 3 * N + 2 * (N * (N - 1) // 2) + N
    state = 3 * (force + hess) + 4 * 2 * N + 3 * 2 * N
    vec = 3 * (2 * N * N) + 3 * 2 * N
    per = state + m_s * vec
    if ld:
        per += (2 * N - 1) + 1 + 2
    ck = m_s * (2 * D - 1 + D + 1)
    if sali:
        ck += 2 * (D + 2 * D - 1)
    if energy:
        ck += 6 * N + 2 * (N * (N - 1) // 2) + 4
    return per + ck / K


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def emit(args, metric, value, unit, elapsed, dtype, config, roofline, cpu, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": elapsed / max(args.steps, 1) * 1e3,
            "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu}


def advance_timed(e, n_steps, spl, stream, torch, log, label=None, sync_every=50):
    """Advance an ensemble to its last step in launches of spl steps, with
    HIP events around each launch on the stream it runs on.  With a label,
    every sync_every launches the stream is drained and the count printed
    (a progress line from the work itself for long runs)."""
    s, k = 0, 0
    total = (n_steps + spl - 1) // spl
    while s < n_steps:
        nxt = min(s + spl, n_steps)
        if log is not None:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            e.advance(nxt)
            b.record(stream)
            log.append((a, b, nxt - s))
        else:
            e.advance(nxt)
        s = nxt
        k += 1
        if label and k % sync_every == 0 and k < total:
            stream.synchronize()
            progress(f"{label}: {k}/{total} launches done")


def bench_fput(args, P, chx, torch, dev):
    """FPU-beta chains, N = 8 and N = 16, 65,536 orbits each (energy 1 per
    mass, random mode amplitudes), 3N deviation vectors per orbit: the 2N
    Lyapunov vectors (modified Gram-Schmidt every 10 steps) and N GALI/SALI
    vectors, dt = 0.02."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 2000.0
    dt, K, n = 0.02, 10, 65536
    n_steps = int(round(T / dt))
    spl = min(args.steps_per_launch or 10000, n_steps)
    stream = torch.cuda.current_stream()
    ind = chx.IND_SALI | chx.IND_GALI | chx.IND_LYAP | chx.IND_ENERGY
    x0s = {}
    for N in (8, 16):
        u = torch.as_tensor(S.fput_mode_draws(1003 + N, n), device=dev)
        x0s[N] = P.ic_fput_modes(P.fput(N), u)
    logs = {8: [], 16: []}
    last = {}

    def one_pass(record):
        for N in (8, 16):
            progress(f"fput: N={N}, {n} orbits, T={T:g}")
            e = P.Ensemble(P.fput(N), x0s[N], steps_per_launch=spl, dt=dt, T=T, indicators=ind,
                           gali_kmax=N, n_lyap=2 * N, renorm_every=K, seed=1003,
                           outputs=("status", "lyap", "gali"))
            advance_timed(e, n_steps, spl, stream, torch, logs[N] if record else None,
                          label=f"fput N={N}")
            last[N] = e.results()
            e.close()

    for _ in range(args.warmup):
        one_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_pass(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = 2 * n * n_steps * args.steps / elapsed
    per_n = {}
    checks = {}
    for N in (8, 16):
        fps = model_flops_fput(N, 2 * N, N, K)
        full = [a.elapsed_time(b) for a, b, k in logs[N] if k == spl]
        ms = float(np.mean(full))
        per_n[N] = dict(fps=fps, fps_exec=flops_per_step_fput(N, N, 2 * N, False, True, True, K),
                        ms=ms, achieved=fps * n * spl / (ms * 1e-3), launches=len(full))
        # on every orbit: the exponents of a Hamiltonian flow sum to zero;
        # GALI_k lies in [0, 1] and does not grow with k
        st = last[N]["status"].cpu().numpy()
        ly = last[N]["lyap"].cpu().numpy()[st == 0]
        ga = last[N]["gali"].cpu().numpy()[st == 0]
        checks[N] = {"orbits_ok": int((st == 0).sum()), "orbits_stopped": int((st != 0).sum()),
                     "max_abs_lyap_sum": float(np.max(np.abs(ly.sum(axis=1)))),
                     "gali_outside_0_1": int(np.sum((ga < 0) | (ga > 1 + 1e-12))),
                     "gali_increasing_in_k": int(np.sum(ga[:, 1:] > ga[:, :-1] * (1 + 1e-9))),
                     "gali_N_median": float(np.median(ga[:, -1]))}
    r = per_n[16]
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        cT = args.cpu_T if args.cpu_T != 1e4 else 2000.0
        tot, el = 0, 0.0
        for N in (8, 16):
            m = 32
            xs = O.fput_ic(O.fput(N), S.fput_mode_draws(1003 + N, m))
            w0 = S.deviation_vectors(1003, m, N, 2 * N)
            run = O.Run(dt=dt, T=cT, indicators=ind, gali_kmax=N, n_lyap=2 * N, K=K)
            t1 = time.perf_counter()
            O.integrate(O.fput(N), xs, run, w0=w0, threads=threads)
            el += time.perf_counter() - t1
            tot += m * int(round(cT / dt))
        nproc, avail, model = host_cpu()
        cpu = {"value": tot / el, "unit": "orbit-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"32 orbits per N (8 and 16), T={cT:g}, same vectors and "
                         f"checkpoints ({tot:.3g} orbit-steps, "
                         f"{el:.1f} s)",
               "host": {"logical_cpus": nproc, "cpus_available": avail, "model": model}}
    return emit(args, "FP64 trajectory-steps/s (with tangents)", value, "orbit-steps/s", elapsed,
                "f64", {
                    "workload": f"FPU-beta chains N=8 and N=16 (k=1, beta=1), 65536 orbits each, "
                                f"3N deviation vectors (2N Lyapunov by MGS/10 + N GALI), "
                                f"dt={dt}, T={T:g}",
                    "orbits": 2 * n, "steps_per_orbit": n_steps, "steps_per_launch": spl,
                    "per_N": {str(N): {"kernel": ("chx::fput_row_kernel<16, 3, 1, 1, true>" if N == 16
                                                  else "chx::fput_rowpair_kernel<8>"),
                                       "flops_per_orbit_step": v["fps"],
                                       "flops_per_orbit_step_executed": v["fps_exec"],
                                       "launch_ms": v["ms"],
                                       "tflops": v["achieved"] / 1e12,
                                       "frac": v["achieved"] / PEAK_FP64,
                                       "checks": checks[N]}
                              for N, v in per_n.items()}},
                {"bound": "alu", "achieved": r["achieved"] / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": r["achieved"] / PEAK_FP64, "traffic": None,
                 "kernel": "chx::fput_row_kernel<16, 3, 1, 1, true>", "flops_per_orbit_step": r["fps"],
                 "flops_per_orbit_step_executed": r["fps_exec"],
                 "launch_ms": r["ms"], "launches_timed": r["launches"]}, cpu)


def bench_dop853(args, P, chx, torch, dev):
    """The headline Henon-Heiles grids (1024^2 section points at E = 0.125
    and E = 1/6, SALI + GALI_2 + 4 Lyapunov vectors + LD + energy, dt = 0.01)
    integrated with the fixed-step DOP853 kernels; T = 200 by default."""
    import numpy as np

    import seeded_inputs as S
    energies = (0.125, 1.0 / 6.0)
    n_side = args.grid
    dt, T, K = 0.01, args.T or 200.0, 10
    ind = chx.IND_SALI | chx.IND_GALI | chx.IND_LYAP | chx.IND_LD | chx.IND_ENERGY
    opts = dict(dt=dt, T=T, indicators=ind, gali_kmax=2, n_lyap=4, renorm_every=K,
                seed=1002, escape_r2=4.0, block_size=args.block, integrator="dop853")
    n_steps = int(round(T / dt))
    spl = min(args.steps_per_launch or 5000, n_steps)
    stream = torch.cuda.current_stream()
    xs, ms = [], []
    for E in energies:
        x, m = P.grid_hh_section(E, n_side, n_side, device=dev)
        xs.append(x)
        ms.append(m)
    x0, mask = torch.cat(xs), torch.cat(ms)
    log = []
    n_active = 0

    def one_pass(record):
        nonlocal n_active
        progress(f"dop853: {n_side}^2 x 2 grids, T={T:g}")
        e = P.Ensemble(P.henon_heiles(), x0, mask=mask, steps_per_launch=spl,
                       outputs=("status", "label", "lyap"), **opts)
        advance_timed(e, n_steps, spl, stream, torch, log if record else None)
        out = e.results()
        n_active = e.info()[2]
        e.close()
        return out

    for _ in range(args.warmup):
        one_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = one_pass(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = n_active * n_steps * args.steps / elapsed
    fps = flops_per_step_dop853(2, 2, 4, True, True, True, K)
    full = [a.elapsed_time(b) for a, b, k in log if k == spl]
    ms_avg = float(np.mean(full))
    achieved = fps * n_active * spl / (ms_avg * 1e-3)
    lab = out["label"].cpu().numpy()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        m, cT = 2048, 150.0
        tot, el = 0, 0.0
        for E in energies:
            xg, mg = O.hh_grid(E, n_side, n_side)
            act = np.flatnonzero(mg)
            idx = act[np.linspace(0, len(act) - 1, m // 2).astype(int)]
            w0 = np.concatenate([S.deviation_vectors(1002, 1, 2, 4, first_ic=int(i))
                                 for i in idx])
            run = O.Run(dt=dt, T=cT, indicators=ind, gali_kmax=2, n_lyap=4, K=K,
                        escape_r2=4.0, integrator=O.INT_DOP853)
            t1 = time.perf_counter()
            O.integrate(O.henon_heiles(), xg[idx], run, w0=w0, threads=threads)
            el += time.perf_counter() - t1
            tot += len(idx) * int(round(cT / dt))
        cpu = {"value": tot / el, "unit": "orbit-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{m} strided grid orbits (both energies), T={cT:g} "
                         f"({tot:.3g} orbit-steps, {el:.1f} s)"}
    return emit(args, "FP64 trajectory-steps/s (with tangents)", value, "orbit-steps/s", elapsed,
                "f64", {
                    "workload": f"henon-heiles {n_side}x{n_side} section grids at E=0.125 and "
                                f"E=1/6, fixed-step DOP853, dt={dt}, T={T:g}, SALI+GALI_2+4 "
                                "Lyapunov (MGS/10)+LD(p=0.5, integrated as a component)+energy",
                    "orbits": int(n_active), "steps_per_orbit": n_steps,
                    "deviation_vectors": 6, "steps_per_launch": spl,
                    "chaotic_fraction": float(np.mean(lab[lab >= 0] == 1))},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_rk_kernel<SysHH, 6, false>", "flops_per_orbit_step": fps,
                 "launch_ms": ms_avg, "launches_timed": len(full)}, cpu)


def bench_dop853_adaptive(args, P, chx, torch, dev):
    """The adaptive DOP8(5) solver on the Henon-Heiles 1024^2 section grid at
    E = 0.125 (850,874 orbits): two deviation vectors (SALI), LD and energy,
    rtol = atol = 1e-10, first step and checkpoint unit dt = 0.1 (checkpoints
    every K dt = 1), T = 1e4 by default.  Reports labelled ICs/s, the
    accepted and rejected steps, and the same grid with fixed-step Yoshida-4
    at dt = 0.01 for comparison (labels and time)."""
    import numpy as np

    T = args.T or 1e4
    dt, K, tol = 0.1, 10, 1e-10
    ind = chx.IND_SALI | chx.IND_LD | chx.IND_ENERGY
    x0, mask = P.grid_hh_section(0.125, args.grid, args.grid, device=dev)
    n_steps = int(round(T / dt))
    spl = min(args.steps_per_launch or 2000, n_steps)
    stream = torch.cuda.current_stream()
    log = []
    res = {}

    def one_pass(record):
        progress(f"dop853 adaptive: {args.grid}^2 grid, T={T:g}, tol {tol:g}")
        e = P.Ensemble(P.henon_heiles(), x0, mask=mask, steps_per_launch=spl, dt=dt, T=T,
                       indicators=ind, renorm_every=K, seed=1002, integrator="dop853_adaptive",
                       rtol=tol, atol=tol, outputs=("status", "label", "steps", "energy_err"))
        advance_timed(e, n_steps, spl, stream, torch, log if record else None)
        out = e.results()
        res["n_active"] = e.info()[2]
        e.close()
        return out

    for _ in range(args.warmup):
        one_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = one_pass(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_active = res["n_active"]
    value = n_active * args.steps / elapsed
    m = mask.cpu().numpy().astype(bool)
    steps = out["steps"].cpu().numpy()[m]
    lab = out["label"].cpu().numpy()[m]
    acc, rej = int(steps[:, 0].sum()), int(steps[:, 1].sum())
    kernel_s = sum(a.elapsed_time(b) for a, b, _ in log) * 1e-3 / args.steps
    fpa = flops_per_attempt_dop853(2, 2, 0, True)
    ck = n_active * (n_steps // K) * checkpoint_flops_hh(2, 2, 0, True, True)
    achieved = ((acc + rej) * fpa + ck) / kernel_s
    # the same grid with fixed-step Yoshida-4 at dt = 0.01
    progress("fixed-step Yoshida-4 on the same grid for comparison")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ref = P.integrate_ensemble(P.henon_heiles(), x0, mask=mask, dt=0.01, T=T, indicators=ind,
                               seed=1002, outputs=("label",))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    rlab = ref["label"].cpu().numpy()[m]
    cpu = None
    if not args.no_cpu_baseline:
        import seeded_inputs as S
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        xg, mg = O.hh_grid(0.125, args.grid, args.grid)
        act = np.flatnonzero(mg)
        ns, cT = 2048, 2000.0
        idx = act[np.linspace(0, len(act) - 1, ns).astype(int)]
        w0 = np.concatenate([S.deviation_vectors(1002, 1, 2, 4, first_ic=int(i)) for i in idx])
        run = O.Run(dt=dt, T=cT, indicators=ind, K=K, integrator=O.INT_DOP853_ADAPTIVE,
                    rtol=tol, atol=tol)
        t2 = time.perf_counter()
        O.integrate(O.henon_heiles(), xg[idx], run, w0=w0, threads=threads)
        el = time.perf_counter() - t2
        cpu = {"value": ns * (cT / T) / el, "unit": "ICs/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} strided grid orbits to T={cT:g} ({el:.1f} s), scaled to T={T:g}"}
    return emit(args, "labelled ICs/s (adaptive DOP8(5))", value, "ICs/s", elapsed, "f64", {
        "workload": f"henon-heiles {args.grid}x{args.grid} section grid at E=0.125, adaptive "
                    f"DOP8(5) rtol=atol={tol:g}, first step {dt}, checkpoints every {K * dt:g}, "
                    f"T={T:g}, SALI (2 vectors)+LD+energy",
        "orbits": int(n_active), "accepted_steps_per_orbit": acc / n_active,
        "rejected_steps_per_orbit": rej / n_active,
        "max_energy_error": float(out["energy_err"].cpu().numpy()[m].max()),
        "kernel_s": kernel_s, "chaotic_fraction": float(np.mean(lab == 1)),
        "yoshida4_dt0.01_s": plain_s, "yoshida4_ICs_per_s": n_active / plain_s,
        "label_agreement_vs_yoshida4": float(np.mean(lab == rlab))},
        {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
         "frac": achieved / PEAK_FP64, "traffic": None,
         "kernel": "chx::lane_rka_kernel<SysHH, 2, false>", "flops_per_attempt": fpa,
         "launch_ms": None, "launches_timed": len(log)}, cpu)


def bench_batched(args, P, chx, torch, dev):
    """The persistent batched form: 2^20 Henon-Heiles orbits (seeded uniform
    accessible section points, E = 0.125), 2^18 coupled-quartic orbits
    (N = 3, eps = 0.1, E = 1) and 2^16 FPU-beta N = 16 orbits in one
    persistent launch sequence, two deviation vectors each, early exit at the
    first checkpoint with SALI < 1e-8, T = 1e5 by default; against three
    plain launches of the same work (one per system, early exit on), and
    each system alone through the batched form.  value = labelled ICs/s of
    the mixed batched run."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 1e5
    y, py = S.section_points(1004, 1400000)
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev),
                               torch.as_tensor(py, device=dev))
    xh = x[m == 1][: 1 << 20].contiguous()
    xq = P.ic_quartic(P.quartic(3, 0.1), torch.as_tensor(S.quartic_draws(1005, 1 << 18),
                                                          device=dev))
    xf = P.ic_fput_modes(P.fput(16), torch.as_tensor(S.fput_mode_draws(1006, 1 << 16),
                                                      device=dev))
    items = [dict(sys=P.henon_heiles(), x0=xh, dt=0.01, T=T),
             dict(sys=P.quartic(3, 0.1), x0=xq, dt=0.01, T=T),
             dict(sys=P.fput(16), x0=xf, dt=0.02, T=T)]
    names = ["henon-heiles", "quartic-3", "fput-16"]
    n_orbits = sum(int(it["x0"].shape[0]) for it in items)
    ind = chx.IND_SALI | chx.IND_ENERGY
    kw = dict(indicators=ind, seed=1004, early_exit=True, sali_threshold=1e-8,
              steps_per_launch=args.steps_per_launch, block_size=args.block)
    outs_keys = ("status", "label", "t_end")
    fps = [model_flops_hh(2, 0, False, True, 10), model_flops_quartic(2),
           model_flops_fput(16, 0, 2, 10)]
    progress(f"batched: {n_orbits} orbits, T={T:g}")
    for _ in range(args.warmup):
        P.integrate_batched(items, outputs=outs_keys, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        outs, stats = P.integrate_batched(items, outputs=outs_keys, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"batched: {elapsed / args.steps:.2f} s per pass; plain launches")
    steps_exec = [int(v) for v in stats["orbit_steps"][:3]]
    kern_s = stats["integrate_ms"] * 1e-3
    flops = sum(f * s for f, s in zip(fps, steps_exec))
    achieved = flops / kern_s
    # three plain launches of the same work; their useful orbit-steps are
    # the steps each orbit actually integrated (t_end / dt)
    plain_s, plain_frac, ref = [], [], []
    for i, it in enumerate(items):
        t1 = time.perf_counter()
        r = P.integrate_ensemble(it["sys"], it["x0"], dt=it["dt"], T=it["T"], outputs=outs_keys,
                                 indicators=ind, seed=1004 + i, early_exit=True,
                                 sali_threshold=1e-8)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        ref.append(r)
        plain_s.append(el)
        useful = float(torch.round(r["t_end"] / it["dt"]).sum())
        plain_frac.append(fps[i] * useful / el / PEAK_FP64)
        progress(f"plain {names[i]}: {el:.2f} s")
    plain = sum(plain_s)
    agree = [float((a["label"] == b["label"]).float().mean()) for a, b in zip(outs, ref)]
    # each system alone through the batched form
    alone = []
    for i, it in enumerate(items):
        t1 = time.perf_counter()
        _, st1 = P.integrate_batched([it], outputs=outs_keys, **dict(kw, seed=1004 + i))
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        s1 = int(st1["orbit_steps"][0])
        alone.append({"seconds": el, "integrate_s": st1["integrate_ms"] * 1e-3,
                      "frac": fps[i] * s1 / (st1["integrate_ms"] * 1e-3) / PEAK_FP64,
                      "threads_per_block": st1["threads_per_block"]})
        progress(f"batched {names[i]} alone: {el:.2f} s")
    value = n_orbits * args.steps / elapsed
    exited = [int((o["status"] == 4).sum()) for o in outs]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batched(args, items, outs, names, T)
    return emit(args, "labelled ICs/s (persistent batched form)", value, "ICs/s", elapsed, "f64", {
        "workload": f"2^20 Henon-Heiles (E=0.125) + 2^18 quartic N=3 + 2^16 FPU-beta N=16, two "
                    f"deviation vectors, early exit at SALI<1e-8, dt 0.01/0.01/0.02, T={T:g}",
        "orbits": n_orbits, "exited_early": exited,
        "executed_orbit_steps": steps_exec,
        "executed_orbit_steps_per_s": sum(steps_exec) / kern_s,
        "threads_per_block": stats["threads_per_block"], "blocks": stats["blocks"],
        "launches": stats["launches"], "steps_per_launch": stats["steps_per_launch"],
        "plain_seconds_per_system": plain_s, "plain_three_launches_s": plain,
        "plain_ICs_per_s": n_orbits / plain,
        "speedup_vs_plain": plain / (elapsed / args.steps),
        "label_agreement_vs_plain": agree,
        "per_system": {names[i]: {"plain_frac": plain_frac[i], "batched_alone": alone[i],
                                  "flops_per_orbit_step": fps[i]} for i in range(3)}},
        {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
         "kernel": "chx::batched_kernel", "flops_per_orbit_step": fps,
         "launch_ms": stats["integrate_ms"] / max(stats["launches"], 1),
         "launches_timed": stats["launches"]}, cpu)


def cpu_baseline_batched(args, items, outs, names, T):
    """The oracle on a strided sample of each system's orbits (192
    Henon-Heiles, 96 quartic, 24 FPU-16), early exit on, to the same T: its
    rate in executed orbit-steps/s, and the sample's labels against the
    batched form's."""
    import numpy as np

    import seeded_inputs as S
    from oracle import oracle as O
    nproc, avail, model = host_cpu()
    threads = max(1, min(HOST_SHARE, avail))
    osys = [O.henon_heiles(), O.quartic(3, 0.1), O.fput(16)]
    counts = [192, 96, 24]
    tot, el, agree, per = 0, 0.0, 0, {}
    for i, it in enumerate(items):
        n = int(it["x0"].shape[0])
        idx = np.linspace(0, n - 1, counts[i]).astype(int)
        xs = it["x0"].cpu().numpy()[idx]
        D = xs.shape[1]
        # the library's deviation vectors for these orbits (the batched form
        # draws them from seed + item index)
        w0 = np.stack([S.deviation_vectors(1004 + i, 1, 2, D, first_ic=int(k))[0] for k in idx])
        run = O.Run(dt=it["dt"], T=T, indicators=O.IND_SALI | O.IND_ENERGY, K=10,
                    early_exit=True, sali_threshold=1e-8)
        t1 = time.perf_counter()
        o = O.integrate(osys[i], xs, run, w0=w0, threads=threads)
        d = time.perf_counter() - t1
        el += d
        steps = float(np.round(o["t_end"] / it["dt"]).sum())
        tot += steps
        lab = outs[i]["label"].cpu().numpy()[idx]
        agree += int((lab == o["label"]).sum())
        per[names[i]] = {"orbits": counts[i], "seconds": d,
                         "label_agreement": float((lab == o["label"]).mean())}
    return {"value": tot / el, "unit": "orbit-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"192 Henon-Heiles + 96 quartic + 24 FPU-16 orbits strided over the "
                      f"workload, early exit, T={T:g} ({tot:.3g} executed orbit-steps, {el:.1f} s)",
            "label_agreement_with_batched": agree / sum(counts), "per_system": per,
            "host": {"logical_cpus": nproc, "cpus_available": avail, "model": model}}


def bench_gate(args, P, chx, torch, dev):
    """The learned gate against the plain form on the Henon-Heiles E = 0.125
    2048x2048 section grid: training labels from 4,194,304 seeded uniform
    accessible section points integrated to T = 1e4 (features at t = 200),
    training on the GPU, then gate + fallback vs the plain integration of the
    test grid (labels by SALI < 1e-8)."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 1e4
    dt, t_gate, conf_min = 0.01, 200.0, 0.98
    n_train = 1 << 22
    ind = chx.IND_SALI | chx.IND_LD
    kw = dict(dt=dt, T=T, indicators=ind, seed=1005)
    s_gate = int(round(t_gate / dt))
    y, py = S.section_points(1005, int(n_train * 1.35))
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev),
                               torch.as_tensor(py, device=dev))
    xt = x[m == 1][:n_train].contiguous()
    assert xt.shape[0] == n_train
    progress(f"gate: labelling {n_train} training orbits to T={T:g}")
    t0 = time.perf_counter()
    e = P.Ensemble(P.henon_heiles(), xt, **kw)
    e.advance(s_gate)
    r = e.results(("ld", "ln_growth"))
    feat = P.gate_features(xt, r["ld"], r["ln_growth"], t_gate)
    e.advance()
    lab = e.results(("label",))["label"]
    e.close()
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    progress(f"gate: labels done in {t_label:.1f} s; training")
    g = P.Gate(1005)
    t0 = time.perf_counter()
    epochs = args.gate_epochs
    losses = g.train(feat, lab, epochs=epochs, batch=4096, lr=1e-3, seed=1005)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    progress(f"gate: trained in {t_train:.1f} s, epoch losses {[round(float(v), 4) for v in losses]}")
    xg, mg = P.grid_hh_section(0.125, 2048, 2048, device=dev)
    n_test = int(mg.sum())
    for _ in range(args.warmup):
        g.classify(P.henon_heiles(), xg, mg, t_gate=t_gate, conf_min=conf_min, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, st = g.classify(P.henon_heiles(), xg, mg, t_gate=t_gate, conf_min=conf_min, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"gate: classify {elapsed / args.steps:.2f} s per pass, {st}; plain run")
    t0 = time.perf_counter()
    ref = P.integrate_ensemble(P.henon_heiles(), xg, mask=mg, outputs=("label",), **kw)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    act = mg == 1
    agree = float((out["label"][act] == ref["label"][act]).float().mean())
    gated = out["source"] == 2
    acc_gated = float((out["label"][gated] == ref["label"][gated]).float().mean()) \
        if int(gated.sum()) else float("nan")
    value = n_test * args.steps / elapsed
    # integration kernel of the gated run: every orbit to t_gate, the
    # unconfident ones on to T (no early exit, no escapes at this energy)
    n_total = int(round(T / dt))
    steps_exec = st["n_active"] * s_gate + st["n_fallback"] * (n_total - s_gate)
    fps = flops_per_step(2, 2, 0, True, False, True, 10)
    kern_s = (st["ms_gate"] + st["ms_fallback"]) * 1e-3
    achieved = fps * steps_exec / kern_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
            "kernel": "chx::lane_kernel<SysHH, 2, false, 2>", "flops_per_orbit_step": fps,
            "launch_ms": None, "launches_timed": None}
    # the perceptron's training against the BF16 matrix peak: the products'
    # algorithmic flops over the whole training time (every kernel of the
    # pass and the gaps between launches included)
    mlp_fl = mlp_train_flops_per_row() * n_train * epochs
    roof_mlp = {"bound": "mfma", "achieved": mlp_fl / t_train / 1e12,
                "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                "frac": mlp_fl / t_train / PEAK_BF16, "traffic": None,
                "kernel": "chx::train_rows_kernel + chx::gemm_tile_kernel (training pass, all kernels)",
                "flops_per_row_epoch": mlp_train_flops_per_row(),
                "executed_flops_per_row_epoch": mlp_train_flops_per_row(True),
                "time_basis": "whole training call"}
    return emit(args, "labelled ICs/s (learned gate + fallback)", value, "ICs/s", elapsed,
                "f64+bf16", {
                    "workload": f"Henon-Heiles E=0.125 2048x2048 section grid, labels by SALI<1e-8 "
                                f"at T={T:g} (dt={dt}); gate at t={t_gate:g}, confidence >= "
                                f"{conf_min}; trained on {n_train} seeded accessible points",
                    "orbits": n_test, "plain_s": t_plain, "plain_ICs_per_s": n_test / t_plain,
                    "speedup_vs_plain": t_plain / (elapsed / args.steps),
                    "agreement_vs_plain": agree, "accepted_accuracy": acc_gated,
                    "fallback_fraction": st["n_fallback"] / max(st["n_active"], 1),
                    "accepted": st["n_accepted"], "fallback": st["n_fallback"],
                    "stopped_before_gate": st["n_early"],
                    "ms_gate_integration": st["ms_gate"], "ms_features_inference": st["ms_infer"],
                    "ms_fallback": st["ms_fallback"],
                    "label_generation_s": t_label, "train_s": t_train, "epochs": epochs,
                    "epoch_loss": [float(v) for v in losses],
                    "train_chaotic_fraction": float((lab == 1).float().mean()),
                    "roofline_mlp_training": roof_mlp},
                roof, None)


def bench_sweep(args, P, chx, torch, dev):
    """Time per orbit against the number of orbits integrated together (the
    shape of the paper's timing figures): Henon-Heiles at E = 0.125, seeded
    accessible section points, SALI (two vectors) + LD, dt = 0.01, T = 200,
    ensembles of 2^8 .. 2^22 orbits; the value is the largest ensemble's
    orbit-steps/s."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 200.0
    dt = 0.01
    n_steps = int(round(T / dt))
    y, py = S.section_points(1001, int((1 << 22) * 1.35))
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev),
                               torch.as_tensor(py, device=dev))
    xa = x[m == 1][: 1 << 22].contiguous()
    ind = chx.IND_SALI | chx.IND_LD
    stream = torch.cuda.current_stream()
    rows = []
    for k in range(8, 23, 2):
        n = 1 << k
        xs = xa[:n].contiguous()
        reps = max(1, min(20, (1 << 18) // n))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        P.integrate_ensemble(P.henon_heiles(), xs, dt=dt, T=T, indicators=ind, seed=1001,
                             outputs=("label",))
        e0.record(stream)
        for _ in range(reps):
            P.integrate_ensemble(P.henon_heiles(), xs, dt=dt, T=T, indicators=ind, seed=1001,
                                 outputs=("label",))
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rows.append({"orbits": n, "ms": ms, "us_per_orbit": ms * 1e3 / n,
                     "orbit_steps_per_s": n * n_steps / (ms * 1e-3)})
        progress(f"sweep: {n} orbits, {ms:.2f} ms, {ms * 1e3 / n:.4f} us per orbit")
    fps = flops_per_step(2, 2, 0, True, False, True, 10)
    best = rows[-1]
    achieved = fps * best["orbit_steps_per_s"]
    return emit(args, "FP64 trajectory-steps/s (with tangents)", best["orbit_steps_per_s"],
                "orbit-steps/s", best["ms"] * 1e-3 * args.steps, "f64", {
                    "workload": f"henon-heiles E=0.125 seeded accessible section points, "
                                f"SALI (2 vectors) + LD, dt={dt}, T={T:g}, ensembles of "
                                f"2^8..2^22 orbits (each call includes set-up and results)",
                    "sweep": rows},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_kernel<SysHH, 2, false, 2>", "flops_per_orbit_step": fps,
                 "launch_ms": None, "launches_timed": None}, None)


def dp_angle_grid(k):
    """2^k double-pendulum states from rest: cell centres of a
    2^ceil(k/2) x 2^floor(k/2) grid of (theta_1, theta_2) over (-pi, pi)^2."""
    import numpy as np
    n1, n2 = 1 << ((k + 1) // 2), 1 << (k // 2)
    t1 = -np.pi + (np.arange(n1) + 0.5) * (2 * np.pi / n1)
    t2 = -np.pi + (np.arange(n2) + 0.5) * (2 * np.pi / n2)
    a, b = np.meshgrid(t1, t2, indexing="ij")
    z = np.zeros(a.size)
    return np.stack([a.ravel(), b.ravel(), z, z], axis=1)


def bench_dp(args, P, chx, torch, dev):
    """The double-pendulum timing figure: alpha = sigma = 1, states from rest
    on a grid of angles over (-pi, pi)^2, SALI (two vectors) + energy, final
    time 1e3; time per initial condition against the number integrated
    together (2^8 .. 2^19), with the fixed-step DOP853 (dt = 0.02) and the
    adaptive DOP8(5) (rtol = atol = 1e-11, first step 0.1, checkpoints every
    1): both hold the energy error near 1e-9.  Each point is one whole call (set-up, integration, results).  The
    value is the largest ensemble's fixed-step ICs/s; the roofline is that
    run's integration kernel, timed launch by launch."""
    import numpy as np

    T = args.T or 1e3
    ind = chx.IND_SALI | chx.IND_ENERGY
    legs = {"dop853": dict(dt=0.02, integrator="dop853"),
            "dop853_adaptive": dict(dt=0.1, integrator="dop853_adaptive", rtol=1e-11,
                                    atol=1e-11)}
    sizes = (8, 10, 12, 14, 16, 17, 18, 19)
    sysd = P.double_pendulum(1.0, 1.0)
    stream = torch.cuda.current_stream()
    rows = {k: [] for k in legs}
    extra = {}
    for _ in range(args.warmup):
        x = torch.as_tensor(dp_angle_grid(8), device=dev)
        for leg in legs.values():
            P.integrate_ensemble(sysd, x, T=T, indicators=ind, seed=7, outputs=("label",), **leg)
    torch.cuda.synchronize()
    log = []
    t_all = time.perf_counter()
    for name, leg in legs.items():
        for k in sizes:
            x = torch.as_tensor(dp_angle_grid(k), device=dev)
            n = x.shape[0]
            n_steps = int(round(T / leg["dt"]))
            spl = min(10000, n_steps)
            last = (k == sizes[-1]) and name == "dop853"
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e = P.Ensemble(sysd, x, steps_per_launch=spl, T=T, indicators=ind, seed=7,
                           outputs=("label", "energy_err", "steps") if name != "dop853"
                           else ("label", "energy_err"), **leg)
            advance_timed(e, n_steps, spl, stream, torch, log if last else None)
            out = e.results()
            e.close()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            lab = out["label"].cpu().numpy()
            row = {"ics": n, "s": sec, "us_per_ic": sec * 1e6 / n, "ics_per_s": n / sec,
                   "max_energy_error": float(out["energy_err"].cpu().numpy().max()),
                   "chaotic_fraction": float(np.mean(lab == 1))}
            if "steps" in out:
                st = out["steps"].cpu().numpy()
                row["accepted_steps_per_ic"] = float(st[:, 0].mean())
                row["rejected_steps_per_ic"] = float(st[:, 1].mean())
            rows[name].append(row)
            progress(f"dp {name}: {n} ICs, {sec:.3f} s, {row['us_per_ic']:.3f} us per IC")
    elapsed = time.perf_counter() - t_all
    big = rows["dop853"][-1]
    n_big = big["ics"]
    kernel_s = sum(a.elapsed_time(b) for a, b, _ in log) * 1e-3
    fps = flops_per_step_dop853(2, 2, 0, False, True, True, 10, system="dp")
    achieved = fps * n_big * int(round(T / legs["dop853"]["dt"])) / kernel_s
    cpu = None
    if not args.no_cpu_baseline:
        import seeded_inputs as S
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        xg = dp_angle_grid(sizes[-1])
        ns = 48
        idx = np.linspace(0, len(xg) - 1, ns).astype(int)
        w0 = S.deviation_vectors(7, ns, 2, 4)
        run = O.Run(dt=legs["dop853"]["dt"], T=T, indicators=ind, integrator=O.INT_DOP853)
        t2 = time.perf_counter()
        O.integrate(O.double_pendulum(1.0, 1.0), xg[idx], run, w0=w0, threads=threads)
        el = time.perf_counter() - t2
        cpu = {"value": ns / el, "unit": "ICs/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} strided grid states, fixed-step DOP853 to T={T:g} ({el:.1f} s)"}
    return emit(args, "double-pendulum ICs/s (fixed-step DOP853)", big["ics_per_s"], "ICs/s",
                elapsed, "f64", {
                    "workload": f"double pendulum alpha=sigma=1 from rest on (theta_1, theta_2) "
                                f"grids over (-pi, pi)^2, SALI (2 vectors)+energy, T={T:g}; "
                                "fixed-step DOP853 dt=0.02 and adaptive DOP8(5) rtol=atol=1e-11; "
                                "2^8..2^19 ICs per call (set-up and results included)",
                    "sweep": rows, "kernel_s_largest_fixed": kernel_s},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_rk_kernel<SysDP, 2, false>", "flops_per_orbit_step": fps,
                 "launch_ms": kernel_s * 1e3 / max(len(log), 1), "launches_timed": len(log)},
                cpu)


def bench_fig2(args, P, chx, torch, dev):
    """The Henon-Heiles timing figure: time per IC against the number of ICs
    integrated together (2^8 .. 2^20 seeded accessible section points at
    E = 0.125), two deviation vectors for SALI + energy, final time 1e4, the
    adaptive DOP8(5) at rtol = atol = 1e-10 (first step 0.1, checkpoints
    every 1).  Each point is one whole call.  The value is the largest
    ensemble's ICs/s; the roofline is its integration kernel over attempted
    steps, timed launch by launch."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 1e4
    dt, tol = 0.1, 1e-10
    ind = chx.IND_SALI | chx.IND_ENERGY
    sizes = (8, 10, 12, 14, 16, 18, 20)
    y, py = S.section_points(1001, int((1 << sizes[-1]) * 1.35))
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev),
                               torch.as_tensor(py, device=dev))
    xa = x[m == 1][: 1 << sizes[-1]].contiguous()
    stream = torch.cuda.current_stream()
    leg = dict(dt=dt, integrator="dop853_adaptive", rtol=tol, atol=tol)
    for _ in range(args.warmup):
        P.integrate_ensemble(P.henon_heiles(), xa[:256].contiguous(), T=T, indicators=ind,
                             seed=1001, outputs=("label",), **leg)
    torch.cuda.synchronize()
    rows, log = [], []
    n_steps = int(round(T / dt))
    spl = min(args.steps_per_launch or 20000, n_steps)
    t_all = time.perf_counter()
    for k in sizes:
        xs = xa[: 1 << k].contiguous()
        last = k == sizes[-1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = P.Ensemble(P.henon_heiles(), xs, steps_per_launch=spl, T=T, indicators=ind,
                       seed=1001, outputs=("label", "energy_err", "steps"), **leg)
        advance_timed(e, n_steps, spl, stream, torch, log if last else None)
        out = e.results()
        e.close()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        st = out["steps"].cpu().numpy()
        rows.append({"ics": 1 << k, "s": sec, "us_per_ic": sec * 1e6 / (1 << k),
                     "ics_per_s": (1 << k) / sec,
                     "max_energy_error": float(out["energy_err"].cpu().numpy().max()),
                     "chaotic_fraction": float(np.mean(out["label"].cpu().numpy() == 1)),
                     "accepted_steps_per_ic": float(st[:, 0].mean()),
                     "rejected_steps_per_ic": float(st[:, 1].mean())})
        progress(f"fig2: {1 << k} ICs, {sec:.3f} s, {rows[-1]['us_per_ic']:.3f} us per IC")
        if last:
            attempts = int(st.sum())
    elapsed = time.perf_counter() - t_all
    kernel_s = sum(a.elapsed_time(b) for a, b, _ in log) * 1e-3
    n_big = 1 << sizes[-1]
    fpa = flops_per_attempt_dop853(2, 2, 0, False)
    ck = n_big * (n_steps // 10) * checkpoint_flops_hh(2, 2, 0, True, True)
    achieved = (attempts * fpa + ck) / kernel_s
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        ns, cT = 256, min(T, 2000.0)
        xs = xa[: 1 << sizes[-1]].cpu().numpy()
        idx = np.linspace(0, len(xs) - 1, ns).astype(int)
        w0 = np.concatenate([S.deviation_vectors(1001, 1, 2, 4, first_ic=int(i)) for i in idx])
        t2 = time.perf_counter()
        O.integrate(O.henon_heiles(), xs[idx], O.Run(dt=dt, T=cT, indicators=ind,
                                                     integrator=O.INT_DOP853_ADAPTIVE,
                                                     rtol=tol, atol=tol),
                    w0=w0, threads=threads)
        el = time.perf_counter() - t2
        cpu = {"value": ns * (cT / T) / el, "unit": "ICs/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} strided ICs of the largest ensemble to T={cT:g} ({el:.1f} s), "
                         f"scaled to T={T:g}"}
    return emit(args, "Henon-Heiles ICs/s (adaptive DOP8(5), SALI)", rows[-1]["ics_per_s"],
                "ICs/s", elapsed, "f64", {
                    "workload": f"henon-heiles E=0.125 seeded accessible section points, SALI "
                                f"(2 vectors)+energy, T={T:g}, adaptive DOP8(5) rtol=atol={tol:g}, "
                                f"first step {dt}, checkpoints every 1; 2^8..2^20 ICs per call "
                                "(set-up and results included)",
                    "sweep": rows, "kernel_s_largest": kernel_s},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_rka_kernel<SysHH, 2, false>", "flops_per_attempt": fpa,
                 "launch_ms": kernel_s * 1e3 / max(len(log), 1), "launches_timed": len(log)},
                cpu)


def bench_fig3(args, P, chx, torch, dev):
    """The FPU timing figure: time of one call against the number of degrees
    of freedom, N = 2, 3, .., 16, for 1000 ICs (energy U[0.1, 10] in the two
    lowest normal modes), GALI_4 (four deviation vectors) + energy, final
    time 1e3, with the adaptive DOP8(5) (the figure's solver) at rtol =
    atol = 1e-11 and with Yoshida-4 at dt = 0.0025, both holding the energy
    error near 1e-8, the figure's level (the figure's absolute tolerance
    1e-8 gives 3e-5 here).  The value is ICs/s of the adaptive
    solver at N = 16; the oracle's time per N on a sample stands beside the
    GPU's, as the figure compares GPU and CPU."""
    import numpy as np

    import seeded_inputs as S
    T = args.T or 1e3
    n = 1000
    ind = chx.IND_GALI | chx.IND_ENERGY
    Ns = tuple(range(2, 17))
    legs = {"dop853_adaptive": dict(dt=0.1, integrator="dop853_adaptive", rtol=1e-11,
                                    atol=1e-11),
            "yoshida4": dict(dt=0.0025)}
    stream = torch.cuda.current_stream()
    x0s = {N: P.ic_fput_modes(P.fput(N), torch.as_tensor(S.fput_mode_draws(1003 + N, n),
                                                           device=dev)) for N in Ns}
    for _ in range(args.warmup):
        for leg in legs.values():
            P.integrate_ensemble(P.fput(2), x0s[2], T=min(T, 10.0), indicators=ind,
                                 gali_kmax=4, seed=1003, outputs=("gali",), **leg)
    torch.cuda.synchronize()
    rows = {k: [] for k in legs}
    log = []
    t_all = time.perf_counter()
    for name, leg in legs.items():
        n_steps = int(round(T / leg["dt"]))
        spl = min(args.steps_per_launch or 100000, n_steps)
        for N in Ns:
            last = N == Ns[-1] and name == "dop853_adaptive"
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs = ("gali", "energy_err", "steps") if name != "yoshida4" else ("gali", "energy_err")
            e = P.Ensemble(P.fput(N), x0s[N], steps_per_launch=spl, T=T, indicators=ind,
                           gali_kmax=4, seed=1003, outputs=outs, **leg)
            advance_timed(e, n_steps, spl, stream, torch, log if last else None)
            out = e.results()
            e.close()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            g4 = out["gali"].cpu().numpy()[:, 2]
            row = {"N": N, "s": sec,
                   "max_energy_error": float(out["energy_err"].cpu().numpy().max()),
                   "median_log10_gali4": float(np.median(np.log10(np.maximum(g4, 1e-300))))}
            if "steps" in out:
                st = out["steps"].cpu().numpy()
                row["accepted_steps_per_ic"] = float(st[:, 0].mean())
                row["rejected_steps_per_ic"] = float(st[:, 1].mean())
                if last:
                    attempts = int(st.sum())
            rows[name].append(row)
            progress(f"fig3 {name}: N={N}, {n} ICs, {sec:.3f} s")
    elapsed = time.perf_counter() - t_all
    kernel_s = sum(a.elapsed_time(b) for a, b, _ in log) * 1e-3
    # roofline of the adaptive N = 16 kernel over attempted steps: the state
    # and four vectors' DOP853 stages (per stage: 12 spring evaluations and
    # stiffnesses as in flops_per_step_fput, 8N per vector stage for the
    # tridiagonal product, the stage sums) and the error terms
    D = 32
    sums = 2 * D * sum(DOP853_ROW_NNZ) + D * (len(DOP853_ROW_NNZ) - 1)
    final = 2 * D * DOP853_B_NNZ + D
    force = 6 * 17 + 16 + 4 * 17
    state = sums + 12 * (force + D) + final
    vec = sums + 12 * (3 * 2 * 16 + D) + final
    err = D * 5 * (2 * DOP853_B_NNZ + 2 * 3 + 2 + 2 * 2)
    fpa = state + 4 * vec + err + 8
    achieved = attempts * fpa / kernel_s
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        ns, cT = 16, min(T, 100.0)
        el_tot = 0.0
        for r in rows["dop853_adaptive"]:
            N = r["N"]
            xs = O.fput_ic(O.fput(N), S.fput_mode_draws(1003 + N, ns))
            w0 = S.deviation_vectors(1003, ns, 4, 2 * N)
            t1 = time.perf_counter()
            O.integrate(O.fput(N), xs, O.Run(dt=0.1, T=cT, indicators=O.IND_GALI | O.IND_ENERGY,
                                              gali_kmax=4, integrator=O.INT_DOP853_ADAPTIVE,
                                              rtol=1e-11, atol=1e-11), w0=w0, threads=threads)
            el = time.perf_counter() - t1
            el_tot += el
            # thread-seconds per IC, spread over all threads, for n ICs to T
            per_ic = el * min(threads, ns) / ns
            r["oracle_s_for_1000_ics"] = per_ic * n / threads * (T / cT)
        last_el = rows["dop853_adaptive"][-1]["oracle_s_for_1000_ics"]
        cpu = {"value": n / last_el, "unit": "ICs/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} ICs per N to T={cT:g} with the adaptive solver on {threads} "
                         f"threads ({el_tot:.1f} s), scaled to 1000 ICs and T={T:g}; the value "
                         "is N=16"}
    big = rows["dop853_adaptive"][-1]
    return emit(args, "FPU ICs/s at N=16 (GALI_4, adaptive DOP8(5))", n / big["s"], "ICs/s",
                elapsed, "f64", {
                    "workload": f"FPU-beta chains (k=1, beta=1), N=2..16, {n} ICs each, "
                                f"GALI_4 (4 vectors)+energy, T={T:g}; adaptive DOP8(5) "
                                "rtol=atol=1e-11 and Yoshida-4 dt=0.0025; time of each whole call",
                    "per_N": rows, "kernel_s_N16_adaptive": kernel_s},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::fput_crow_rka_kernel<16, 4> (1000 orbits: a small fraction of "
                           "the chip)", "flops_per_attempt": fpa,
                 "launch_ms": kernel_s * 1e3 / max(len(log), 1), "launches_timed": len(log)}, cpu)


CUSTOM_HH_SOURCE = r"""
__device__ double chx_potential(const double *q, const double *prm) {
  return 0.5 * (q[0] * q[0] + q[1] * q[1]) + q[0] * q[0] * q[1] - q[1] * q[1] * q[1] / 3.0;
}
__device__ void chx_force(const double *q, double *F, const double *prm) {
  F[0] = q[0] + 2.0 * q[0] * q[1];
  F[1] = q[1] + q[0] * q[0] - q[1] * q[1];
}
__device__ void chx_hess(const double *q, double *H, const double *prm) {
  H[0] = 1.0 + 2.0 * q[1];
  H[1] = 2.0 * q[0];
  H[2] = 1.0 - 2.0 * q[1];
}
"""


def bench_custom(args, P, chx, torch, dev):
    """The headline workload (Henon-Heiles 1024^2 grids at both energies,
    six vectors, SALI + GALI_2 + Lyapunov + LD + energy, dt = 0.01) with the
    system given as user source (CHX_SYS_CUSTOM, compiled at run time), T =
    1000 by default, beside the built-in system on the same grids: the run-
    time compiled kernels against the library's own."""
    import numpy as np

    T = args.T or 1e3
    dt, K = 0.01, 10
    ind = chx.IND_SALI | chx.IND_GALI | chx.IND_LYAP | chx.IND_LD | chx.IND_ENERGY
    xs, ms = [], []
    for E in (0.125, 1.0 / 6.0):
        x, m = P.grid_hh_section(E, args.grid, args.grid, device=dev)
        xs.append(x)
        ms.append(m)
    x0, mask = torch.cat(xs), torch.cat(ms)
    n_steps = int(round(T / dt))
    spl = min(args.steps_per_launch or 25000, n_steps)
    stream = torch.cuda.current_stream()
    opts = dict(dt=dt, T=T, indicators=ind, gali_kmax=2, n_lyap=4, renorm_every=K, seed=1002,
                escape_r2=4.0)
    res = {}
    t_compile = time.perf_counter()
    P.integrate_ensemble(P.custom(2, CUSTOM_HH_SOURCE), x0[:64].contiguous(), dt=dt, T=0.1,
                         indicators=ind, gali_kmax=2, n_lyap=4, seed=1002, outputs=("status",))
    torch.cuda.synchronize()
    compile_s = time.perf_counter() - t_compile
    for name, sysg in (("custom", P.custom(2, CUSTOM_HH_SOURCE)), ("built-in", P.henon_heiles())):
        log = []
        e = P.Ensemble(sysg, x0, mask=mask, steps_per_launch=spl, outputs=("label",), **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        advance_timed(e, n_steps, spl, stream, torch, log)
        lab = e.results()["label"].cpu().numpy()
        n_act = e.info()[2]
        e.close()
        torch.cuda.synchronize()
        full = [a.elapsed_time(b) for a, b, k in log if k == spl]
        res[name] = dict(s=time.perf_counter() - t0, launch_ms=float(np.mean(full)), labels=lab,
                         n=n_act)
        progress(f"custom: {name} system, {n_act} orbits, T={T:g}: {res[name]['s']:.2f} s")
    fps = flops_per_step(2, 2, 4, True, True, True, K)
    c = res["custom"]
    achieved = fps * c["n"] * spl / (c["launch_ms"] * 1e-3)
    value = c["n"] * n_steps / c["s"]
    agree = float(np.mean(res["custom"]["labels"] == res["built-in"]["labels"]))
    return emit(args, "FP64 trajectory-steps/s (with tangents), user-source system", value,
                "orbit-steps/s", c["s"], "f64", {
                    "workload": f"henon-heiles 1024x1024 section grids at E=0.125 and E=1/6 "
                                f"given as user source (run-time compiled), dt={dt}, T={T:g}, "
                                "SALI+GALI_2+4 Lyapunov+LD+energy; the built-in system beside it",
                    "compile_s_first_call": compile_s,
                    "launch_ms_custom": c["launch_ms"],
                    "launch_ms_builtin": res["built-in"]["launch_ms"],
                    "label_agreement_with_builtin": agree},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_kernel<SysCustom, 6, false, 2> (run-time compiled)",
                 "flops_per_orbit_step": fps, "launch_ms": c["launch_ms"],
                 "launches_timed": None}, None)


def auc(score, label):
    """Area under the ROC curve of score for label 1 against label 0 (ties
    counted half): the probability that a random chaotic orbit scores above
    a random regular one."""
    import numpy as np
    s1, s0 = np.sort(score[label == 1]), np.sort(score[label == 0])
    if len(s1) == 0 or len(s0) == 0:
        return None
    lo = np.searchsorted(s0, s1, side="left")
    hi = np.searchsorted(s0, s1, side="right")
    return float((lo.sum() + 0.5 * (hi - lo).sum()) / (len(s1) * len(s0)))


def bench_ldn(args, P, chx, torch, dev):
    """Chaos indicators from the two-sided LDs of neighbouring orbits on the
    Henon-Heiles section grid at E = 0.125 (1024^2, 850,874 accessible ICs):
    neighbours at +/- 1e-3 along y and p_y, T = 200 forward and backward
    (ten member orbits per IC, LD only, Yoshida-4 at dt = 0.01).  Value =
    ICs/s of the whole call; the indicators are scored against SALI labels
    of the same grid at T = 1e4 (the headline's ground truth, integrated in
    the same run) by the area under the ROC curve and the best single
    threshold's agreement."""
    import numpy as np

    T = args.T or 200.0
    dt, sigma, E = 0.01, 1e-3, 0.125
    n_side = args.grid
    x0, mask = P.grid_hh_section(E, n_side, n_side, device=dev)
    m = mask.cpu().numpy().astype(bool)
    stream = torch.cuda.current_stream()
    kw = dict(dt=dt, T=T, block_size=args.block)

    def one():
        return P.ld_indicators(P.henon_heiles(), x0, sigma, dirs=[1, 3], mask=mask, **kw)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        out = one()
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) * 1e-3 / args.steps
    n_act = int(m.sum())
    value = n_act * args.steps / elapsed
    progress(f"ldn: {n_act} ICs x 10 member orbits, T={T:g}: {elapsed / args.steps:.3f} s per call")
    # ground truth: SALI labels at T = 1e4 on the same grid
    ref = P.integrate_ensemble(P.henon_heiles(), x0, mask=mask, dt=0.01, T=1e4,
                               indicators=chx.IND_SALI, seed=1002, outputs=("label",))
    lab = ref["label"].cpu().numpy()[m]
    st = out["status"].cpu().numpy()[m]
    ok = (st == 0) & (lab >= 0) & (lab <= 1)
    scores = {}
    for k in ("D", "R", "S"):
        v = out[k].cpu().numpy()[m][ok]
        lv = np.log10(np.maximum(v, 1e-300))
        a = auc(lv, lab[ok])
        order = np.argsort(lv)
        ls = lab[ok][order]
        # best threshold: chaotic iff score > t; agreement over all cut points
        chaotic_above = np.concatenate([[0], np.cumsum(ls[::-1])])[::-1]
        regular_below = np.concatenate([[0], np.cumsum(1 - ls)])
        agree = (chaotic_above + regular_below) / len(ls)
        scores[k] = {"auc": a, "best_threshold_agreement": float(agree.max())}
    n_orbits = n_act * 10
    n_steps = int(round(T / dt))
    fps = flops_per_step(2, 0, 0, True, False, False, 10)
    achieved = fps * n_orbits * n_steps / gpu_s
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        xg, mg = O.hh_grid(E, n_side, n_side)
        act = np.flatnonzero(mg)
        ns = 512
        idx = act[np.linspace(0, len(act) - 1, ns).astype(int)]
        t2 = time.perf_counter()
        O.ld_indicators(O.henon_heiles(), xg[idx], O.Run(dt=dt, T=T, indicators=O.IND_LD),
                        [1, 3], sigma, threads=threads)
        el = time.perf_counter() - t2
        cpu = {"value": ns / el, "unit": "ICs/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} strided grid ICs, the same indicators ({el:.1f} s)"}
    return emit(args, "ICs/s (LD indicators from neighbouring orbits)", value, "ICs/s", elapsed,
                "f64", {
                    "workload": f"henon-heiles {n_side}x{n_side} section grid at E=0.125, "
                                f"neighbours +/-{sigma:g} along y and p_y, two-sided LD over "
                                f"[-{T:g}, {T:g}] (10 member orbits per IC, Yoshida-4 dt={dt}); "
                                "D, R, S scored against SALI labels at T=1e4",
                    "ics": n_act, "member_orbits": n_orbits, "gpu_s_per_call": gpu_s,
                    "chaotic_fraction_sali": float(np.mean(lab[ok] == 1)),
                    "scores_log10": scores,
                    "statuses": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}},
                {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                 "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                 "kernel": "chx::lane_kernel<SysHH, 0, false> (whole call, set-up included)",
                 "flops_per_orbit_step": fps, "launch_ms": None, "launches_timed": None},
                cpu)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("hh", "fput", "batched", "gate", "sweep", "dop853",
                                           "dop853_adaptive", "dp", "ldn", "fig2", "fig3",
                                           "custom"),
                    default="hh",
                    help="hh: the headline Henon-Heiles grids (default); fput: FPU-beta "
                         "chains with 3N deviation vectors; batched: the persistent mixed "
                         "form with early exit; gate: the learned gate against the plain "
                         "form; sweep: time per orbit against the ensemble size; dop853: "
                         "the headline grids with the fixed-step DOP853 integrator; "
                         "dop853_adaptive: the adaptive DOP8(5) solver on the E=0.125 grid "
                         "against fixed-step Yoshida-4; dp: the double pendulum's time per "
                         "IC against the ensemble size, fixed and adaptive; ldn: chaos "
                         "indicators from the LDs of neighbouring orbits against SALI labels; "
                         "fig2: Henon-Heiles time per IC against the ensemble size with the "
                         "adaptive solver; fig3: FPU time against the degrees of freedom; "
                         "custom: the headline grids with the system given as user source")
    ap.add_argument("--grid", type=int, default=1024, help="grid side per energy")
    ap.add_argument("--T", type=float, default=None,
                    help="final time (default: 1e4 for hh, gate and batched, 2e3 for fput, "
                         "200 for dop853)")
    ap.add_argument("--steps-per-launch", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="orbits in the oracle sample (strided over the workload)")
    ap.add_argument("--cpu-T", type=float, default=1e4)
    ap.add_argument("--gate-epochs", type=int, default=24,
                    help="training epochs of the gate workload")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this path has no multi-GPU form "
              "(orbits are independent: each GPU would integrate its own contiguous "
              "share of the orbit list and the results would be gathered once at the "
              "end).", file=sys.stderr)
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
    if args.workload != "hh":
        fn = {"fput": bench_fput, "batched": bench_batched, "gate": bench_gate,
              "sweep": bench_sweep, "dop853": bench_dop853,
              "dop853_adaptive": bench_dop853_adaptive, "dp": bench_dp,
              "ldn": bench_ldn, "fig2": bench_fig2, "fig3": bench_fig3,
              "custom": bench_custom}[args.workload]
        print(json.dumps(fn(args, P, chx, torch, dev)), flush=True)
        return
    if args.T is None:
        args.T = 1e4
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
    fps = model_flops_hh(2, 4, True, True, K)
    fps_exec = flops_per_step(2, 2, 4, True, True, True, K)
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
            "kernel": "chx::lane_kernel<SysHH, 6, false, 2>",
            "kernel_code_sha256": kernel_code_hash(),
            "flops_per_orbit_step": fps,
            "flops_per_orbit_step_executed": fps_exec,
            "launch_ms": ms_avg,
            "launches_timed": len(full),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def host_cpu():
    """The host's logical CPU count, the CPUs this process may run on, and
    the CPU model string."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, len(os.sched_getaffinity(0)), model


# A GPU machine gives one GPU's share of its host: 16 CPUs, whatever the count
# of logical CPUs shows; the oracle's thread pool is held to that share.
HOST_SHARE = 16


def cpu_baseline(args, energies, n_side, dt, K):
    """The oracle, as it stands, on this host's cores: a strided sample of the
    workload's orbits (both energies) for T = cpu_T, once on the CPUs of one
    GPU's share of the host and once on one thread (a sixteenth of the
    sample)."""
    import numpy as np

    import seeded_inputs as S
    from oracle import oracle as O
    nproc, avail, model = host_cpu()
    threads = max(1, min(HOST_SHARE, avail))
    xs = []
    for E in energies:
        x0, m = O.hh_grid(E, n_side, n_side)
        xs.append(x0[m == 1])
    x = np.concatenate(xs)
    run = O.Run(dt=dt, T=args.cpu_T, indicators=31, gali_kmax=2, n_lyap=4, K=K, escape_r2=4.0)
    steps = int(round(args.cpu_T / dt))

    def timed(count, nthreads):
        idx = np.linspace(0, len(x) - 1, count).astype(int)
        w0 = S.deviation_vectors(1002, count, 2, 4)
        t0 = time.perf_counter()
        O.integrate(O.henon_heiles(), x[idx], run, w0=w0, threads=nthreads)
        return count * steps, time.perf_counter() - t0

    n, el = timed(args.cpu_sample, threads)
    n1, el1 = timed(max(1, args.cpu_sample // 16), 1)
    return {"value": n / el, "unit": "orbit-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{args.cpu_sample} orbits strided over both grids, T={args.cpu_T:g} "
                      f"({n:.3g} orbit-steps, {el:.1f} s on {threads} threads); one thread: "
                      f"{max(1, args.cpu_sample // 16)} orbits ({n1:.3g} orbit-steps, {el1:.1f} s)",
            "single_thread_value": n1 / el1,
            "host": {"logical_cpus": nproc, "cpus_available": avail, "model": model}}


if __name__ == "__main__":
    main()
