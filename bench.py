#!/usr/bin/env python3
"""Throughput of one gradient evaluation of the joint holotomography objective.

One step = holo_grad on the whole workload: ray sums and exp for every angle,
the four-plane frame stages (forward propagation, residual, adjoint
propagation, probe and object gradients), the transpose of the ray sums, the
probe-gradient finish and the double-precision objective.  Inputs are
synthetic, seeded and already resident in HBM when the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gradient evals/s (fwd+adjoint, object+probe) at 1024², vs plain; HBM GB/s"
PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0           # MI355X published HBM3E bandwidth
FLOP_PER_LERP = 8               # 2 taps x (re, im) x fused multiply-add

# HBM traffic per launch of the ray-sum kernels, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the launches of
# one gradient evaluation), each scaled by what the same counter reads for a
# 1 GiB device-to-device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  The
# figures hold for the kernel sources they were taken on (SHA-256 over
# KERNEL_SOURCES) and the workload they were taken on; after any change to
# those sources, or on another workload, the field reports null.
TRAFFIC = {
    "k_radon_fwd": {"workload": "vol1024_a1800", "fetch_kib": 17815383.81, "write_kib": 508471.91,
                    "fetch_scale": 2.0, "write_scale": 1.0,
                    "sources_sha256": "6b32a6c8213a1a15bec205f27aa2afc6b8740ccca556363f00ff598746146a47"},
    "k_radon_adj": {"workload": "vol1024_a1800", "fetch_kib": 136143410.9, "write_kib": 8388608.0,
                    "fetch_scale": 2.0, "write_scale": 1.0,
                    "sources_sha256": "6b32a6c8213a1a15bec205f27aa2afc6b8740ccca556363f00ff598746146a47"},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources the ray-sum kernels are built from (their bodies and launchers,
# and the shared constants and geometry header).
KERNEL_SOURCES = ("holo_radon.hip", "holo_internal.hpp")


def csrc_sha256():
    """SHA-256 of the ray-sum sources with comments and blank lines removed
    (a change of wording leaves the kernels, and their traffic, as they
    were)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_20304_amd", "csrc", name)) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def traffic_bytes(kernel, workload):
    t = TRAFFIC.get(kernel)
    if t is None or t["workload"] != workload or t["sources_sha256"] != csrc_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def frame_bytes_model(wl, steps):
    """Pass-minimal HBM bytes of the frame stages per timed region: per angle
    one read of psi and one write of h (8 + 8 B/px); per (angle, plane)
    frame the amplitude read (4 B/px) and two row/column exchanges (write +
    read, 16 B/px each)."""
    P = wl.H * wl.W
    per_eval = wl.n_angles * P * (16 + len(wl.mag_rel) * 36)
    return per_eval * steps


_CPU = {}


def _cpu_angle(k):
    """One angle of the oracle sample in a worker process (single-threaded
    NumPy): ray sums and their transpose on the slab, then the four-plane
    frame stage of that angle at full detector size."""
    from oracle import holo_oracle as O
    c = _CPU
    theta = float(c["theta"][k])
    t0 = time.perf_counter()
    p = O.radon(c["u_slab"], theta)
    O.radon_T(p, theta, c["W"])
    t1 = time.perf_counter()
    O.holo2d_gradient(c["psi"], c["q"], c["amp"][c["ks"].index(k)], c["a_ref"], c["mag_rel"],
                      c["m0"], c["fresnel0"])
    return t1 - t0, time.perf_counter() - t1


def _cpu_init():
    from threadpoolctl import threadpool_limits
    _CPU["limits"] = threadpool_limits(1)


def cpu_baseline_child(d):
    """The oracle sample itself, in a process that never touches the GPU
    (started by cpu_baseline): loads the sample from directory `d`, runs its
    angles on a pool of worker processes and prints one JSON line."""
    import multiprocessing as mp
    import platform
    import numpy as np
    meta = json.load(open(os.path.join(d, "meta.json")))
    for name in ("theta", "u_slab", "q", "a_ref", "amp", "mag_rel"):
        _CPU[name] = np.load(os.path.join(d, name + ".npy"))
    _CPU["ks"] = list(meta["ks"])
    _CPU.update({k: meta[k] for k in ("W", "m0", "fresnel0")})
    rng = np.random.default_rng(0)
    _CPU["psi"] = np.exp(1j * rng.uniform(0, 1, (meta["H"], meta["W"])))
    cores = max(1, min(16, len(os.sched_getaffinity(0)), len(_CPU["ks"])))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_cpu_init) as pool:
        times = pool.map(_cpu_angle, _CPU["ks"])
    wall = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        model = platform.processor()
    print(json.dumps({"times": times, "wall": wall, "cores": cores, "cpu": model,
                      "numpy": np.__version__}), flush=True)


def cpu_baseline(wl, u_gpu, q, amp_gpu, amp_ref, slab, n_sample=16):
    """Time the FP64 oracle on a bounded sample of the same workload, on the
    host's cores (one worker process per core, up to 16): `n_sample` angles of
    the strided subset {floor(i N / n_sample)}, each with its ray sums and
    their transpose on a `slab`-slice slab of the volume plus its full
    four-plane frame stage.  The single-core seconds of the sample are scaled
    to a whole evaluation (ray sums x H / slab, angles x N / n_sample) and
    divided by the worker count (angles are independent).  The sample runs
    in a child process that never touches the GPU."""
    import shutil
    import subprocess
    import tempfile
    import numpy as np
    ks = [(i * wl.n_angles) // n_sample for i in range(n_sample)]
    z0 = wl.H // 2 - slab // 2
    d = tempfile.mkdtemp(prefix="holo_cpu_")
    try:
        np.save(os.path.join(d, "theta.npy"), np.asarray(wl.theta, dtype=np.float64))
        np.save(os.path.join(d, "u_slab.npy"), u_gpu[z0:z0 + slab].cpu().numpy())
        np.save(os.path.join(d, "q.npy"), q.astype(np.complex128))
        np.save(os.path.join(d, "a_ref.npy"), amp_ref.astype(np.float64))
        np.save(os.path.join(d, "amp.npy"), np.stack([amp_gpu[k].cpu().numpy() for k in ks])
                .astype(np.float64))
        np.save(os.path.join(d, "mag_rel.npy"), np.asarray(wl.mag_rel, dtype=np.float64))
        json.dump({"ks": ks, "H": wl.H, "W": wl.W, "m0": wl.m0, "fresnel0": wl.fresnel0},
                  open(os.path.join(d, "meta.json"), "w"))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", d],
                           capture_output=True, text=True, check=True)
        out = json.loads(r.stdout.strip().splitlines()[-1])
    finally:
        shutil.rmtree(d, ignore_errors=True)
    times, cores, wall = out["times"], out["cores"], out["wall"]
    t_ray = sum(t[0] for t in times)
    t_frame = sum(t[1] for t in times)
    core_s = (t_ray * (wl.H / slab) + t_frame) * (wl.n_angles / n_sample)
    t_eval = core_s / cores
    log("  oracle sample: %d angles on %d workers in %.1f s wall" % (n_sample, cores, wall))
    return {
        "value": 1.0 / t_eval, "unit": "gradient evals/s", "cores": cores, "kind": "oracle",
        "cpu": out["cpu"], "numpy": out["numpy"],
        "sample": ("%d angles of the strided subset {floor(i %d / %d)}, %d worker processes "
                   "(%.1f s wall): ray sums + transpose on a %d-slice slab (%.1f core-s, "
                   "extrapolated x%d to %d slices) and the 4-plane frame stage at %dx%d "
                   "(%.1f core-s); extrapolated x%d/%d to all angles -> %.0f core-s, %.0f s "
                   "per evaluation on %d cores") %
                  (n_sample, wl.n_angles, n_sample, cores, wall, slab, t_ray, wl.H // slab, wl.H,
                   wl.H, wl.W, t_frame, wl.n_angles, n_sample, core_s, t_eval, cores),
    }


def fourier_bench(wl, u, q, amp, amp_ref, steps, joseph_rate, joseph_F):
    """The same gradient with the Fourier-slice projector (gridding) in place
    of Joseph's ray sums: evaluations per second and the time of its forward
    and transpose kernels.  The two projectors are different discretisations
    of R, so their objectives differ by the discretisation gap (reported)."""
    import torch
    from paper_2407_20304_amd import holo
    plan = holo.Plan.for_workload(wl)
    plan.set_projector("fourier")
    dev = u.device
    F = torch.empty((1,), dtype=torch.float64, device=dev)
    g_u, g_q = torch.empty_like(u), torch.empty_like(q)
    plan.workspace(dev)
    plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=g_u, g_q=g_q)
    torch.cuda.synchronize()
    plan.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=g_u, g_q=g_q)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.timing(False)
    kt = plan.kernel_times()
    res = {"projector": "Fourier-slice gridding (2x oversampled grid, 8-tap kernel)",
           "evals_per_s": steps / elapsed, "ms_per_step": 1000.0 * elapsed / steps,
           "speedup_vs_joseph": (steps / elapsed) / joseph_rate,
           "kernels_ms_per_step": {k: v[0] / steps for k, v in kt.items() if v[1] > 0},
           "objective": F.item(),
           "objective_rel_diff_vs_joseph": abs(F.item() - joseph_F) / abs(joseph_F)}
    plan.close()
    del g_u, g_q
    torch.cuda.empty_cache()
    return res


def plain_bench(wl, u, q, amp, amp_ref, F, g_u, g_q, fused_rate):
    """Time one gradient of the plain unfused form on the same inputs (after
    a warm-up on the first chunk of angles) and compare its outputs with the
    fused library's."""
    import torch
    from paper_2407_20304_amd import plain
    args = (wl.H, wl.W)
    geo = (wl.mag_rel, wl.m0, wl.fresnel0, wl.kappa)
    warm = plain.PlainGrad(*args, wl.theta[:wl.chunk], *geo, chunk=wl.chunk)
    warm.grad(u, q, amp[:wl.chunk], amp_ref)
    torch.cuda.synchronize()
    del warm
    log("plain form: warm-up done; timing one gradient over %d angles" % wl.n_angles)
    pg = plain.PlainGrad(*args, wl.theta, *geo, chunk=wl.chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Fp, gup, gqp = pg.grad(u, q, amp, amp_ref)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log("plain form: %.2f s" % t)

    def rel(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    out = {
        "form": "per-angle plain ray-sum kernels (one thread per ray / voxel, one launch per "
                "angle) + torch ops for every frame step (rocFFT, gather, index_add_), "
                "intermediates materialised per 64-angle chunk, FP32",
        "evals_per_s": 1.0 / t, "ms_per_step": 1000.0 * t, "speedup": fused_rate * t,
        "rel_diff_vs_fused": {"F": abs(Fp.item() - F.item()) / abs(F.item()),
                              "g_u": rel(gup, g_u), "g_q": rel(gqp, g_q)},
    }
    del gup, gqp
    return out


def solver_bench(args, wl, plan, u, amp, amp_ref):
    """Dai-Yuan conjugate gradients at the full workload: iterations per
    second, objective and gradient evaluations per iteration, and the HBM
    rate of the solver's own vector kernels (inner products, x + t eta,
    -g + beta eta, copies) against a pass-minimal byte count."""
    import torch
    q0 = plan.holo_probe_init(amp_ref)
    F, g_u, g_q = plan.holo_grad(u, q0, amp, amp_ref)
    gg = float(torch.linalg.vector_norm(g_u).double() ** 2 + torch.linalg.vector_norm(g_q).double() ** 2)
    step0 = F.item() / gg          # the step that zeroes the linear model of F along -g
    torch.cuda.synchronize()
    log("solver: F0 %.6e, ||g||^2 %.3e, first trial step %.3e" % (F.item(), gg, step0))
    plan.timing(True)
    t0 = time.perf_counter()
    _, _, F_hist, steps, halv = plan.holo_cg(u, q0, amp, amp_ref, args.solver, step0,
                                             in_place=True)
    elapsed = time.perf_counter() - t0
    plan.timing(False)
    kt = plan.kernel_times()
    log("solver: %d iterations in %.3f s, F %s, halvings %s"
        % (args.solver, elapsed, [float(f) for f in F_hist], [int(h) for h in halv]))
    n = u.numel() + q0.numel()
    accepted = [bool(h <= 30) for h in halv]
    trials = sum(min(int(h), 30) + 1 for h in halv)
    # bytes per element (complex64): first direction 16; per iteration the
    # slope dot 16 and 24 per trial point; per accepted step the copies 16,
    # ||g||^2 8, <g, eta> 16 and the new direction 24
    solver_bytes = n * 8 * (2 + sum(2 + 3 * (min(int(h), 30) + 1) + (8 if a else 0)
                                    for h, a in zip(halv, accepted)))
    sms, sn = kt["solver"]
    ev_grad = 1 + int(sum(accepted))
    result = {
        "metric": "CG iterations/s (Dai-Yuan, joint u and q)",
        "value": args.solver / elapsed, "unit": "iterations/s", "n_gpus": 1,
        "iterations": args.solver, "seconds": elapsed, "higher_is_better": True,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": wl.name, "volume": [wl.H, wl.W, wl.W], "n_angles": wl.n_angles,
                   "chunk": wl.chunk, "n_dist": len(wl.mag_rel)},
        "F_hist": [float(f) for f in F_hist], "steps": [float(t) for t in steps],
        "halvings": [int(h) for h in halv],
        "gradient_evals": ev_grad, "objective_evals": trials,
        "solver_kernels": {"ms": sms, "launches": sn, "bytes": solver_bytes,
                           "GBps": solver_bytes / (sms * 1e-3) / 1e9 if sms > 0 else None,
                           "hbm_frac": (solver_bytes / (sms * 1e-3) / 1e9 / PEAK_HBM_GBS)
                           if sms > 0 else None},
        "kernel_ms": {k: v[0] for k, v in kt.items() if v[1] > 0},
    }
    print(json.dumps(result), flush=True)


def batch2d_bench(steps=20, warmup=3):
    """The batched single-angle workload: 96 independent problems with the
    seeded size mix (128 to 512 px, 4 planes, own probe and reference each).
    One call of holo2d_grad evaluates every instance's objective and both
    gradients.  Reports calls per second (HIP events on the launch stream)
    and the HBM rate against the compulsory bytes: psi, q, amp and amp_ref
    read, g_psi and g_q written (8 + 8 + 4 nd + 4 + 8 + 8 bytes per pixel)."""
    import torch
    from paper_2407_20304_amd import holo, synth
    sizes = synth.batch_sizes()
    nd = len(synth.MAG_REL)
    plan = holo.Plan2D(sizes, synth.MAG_REL, synth.M0, synth.FRESNEL0)
    dev = torch.device("cuda:0")
    sd = lambda role, i: synth.seed_of(2, role) + 100 * i
    psi = plan.pack([synth.phase_object_2d(n, sd(4, i)) for i, n in enumerate(sizes)], device=dev)
    q = plan.pack([synth.probe(n, n, sd(5, i)) for i, n in enumerate(sizes)], device=dev)
    amp = plan.pack([synth.synthetic_amplitudes(1, nd, n, n, sd(9, i), device=dev)[0].cpu().numpy()
                     for i, n in enumerate(sizes)], planes=True, device=dev)
    amp_ref = plan.pack([synth.synthetic_amplitudes(1, 1, n, n, sd(9, i) + 500, device=dev)[0, 0]
                         .cpu().numpy() for i, n in enumerate(sizes)], device=dev)
    F = torch.empty(plan.n_inst, dtype=torch.float64, device=dev)
    g_psi, g_q = torch.empty_like(psi), torch.empty_like(q)
    for _ in range(warmup):
        plan.holo2d_grad(psi, q, amp, amp_ref, F=F, g_psi=g_psi, g_q=g_q)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.holo2d_grad(psi, q, amp, amp_ref, F=F, g_psi=g_psi, g_q=g_q)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if not bool(torch.isfinite(F).all()):
        raise RuntimeError("batched objective is not finite")
    # the same call captured once in a HIP graph and replayed: the launch
    # sequence without per-call host work; the replays must reproduce the
    # eager results bit for bit
    F_eager, gp_eager, gq_eager = F.clone(), g_psi.clone(), g_q.clone()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            plan.holo2d_grad(psi, q, amp, amp_ref, F=F, g_psi=g_psi, g_q=g_q)
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    if not (bool((F == F_eager).all()) and bool((g_psi == gp_eager).all())
            and bool((g_q == gq_eager).all())):
        raise RuntimeError("graph replay differs from the eager call")
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    del graph
    T = plan.total
    compulsory = T * (8 + 8 + 4 * nd + 4 + 8 + 8)
    # FFT flops at 5 N log2 N per N-point transform: a propagation D is two
    # 2-D transforms of n^2 points (20 n^2 log2 n); per instance 4 per plane
    # (probe, forward field, its adjoint, probe-gradient adjoint) and 2 for
    # the reference term
    fft_flop = sum((4 * nd + 2) * 20 * n * n * math.log2(n) for n in sizes)
    res = {"workload": "batch96_mixed", "instances": plan.n_inst,
           "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))}, "pixels": T,
           "n_dist": nd, "calls": steps, "ms_per_call": ms, "calls_per_s": 1e3 / ms,
           "ms_per_call_graph": ms_graph,
           "compulsory_bytes": compulsory, "GBps": compulsory / (ms * 1e-3) / 1e9,
           "hbm_frac": compulsory / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "fft_flop": fft_flop, "fft_TFLOPs": fft_flop / (ms * 1e-3) / 1e12}
    plan.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="vol1024_a1800")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slab", type=int, default=32)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy before the timed region "
                         "(a known-size reference for HBM traffic counters)")
    ap.add_argument("--overlap", type=int, choices=(0, 1), default=None,
                    help="run the next chunk's forward ray sums on a second stream during the "
                         "current chunk's frame passes (1) or not (0); default: the plan's")
    ap.add_argument("--fwd-bins", type=int, choices=(8, 16), default=None,
                    help="bins per workgroup of Joseph's forward ray sums (16: 4 angles per "
                         "workgroup, 8: 8 angles); default: the plan's")
    ap.add_argument("--col-tile", type=int, default=None,
                    help="columns per workgroup of the fused column pass (0: the default for "
                         "the detector height, or half of it); default: the plan's")
    ap.add_argument("--tune", action="store_true",
                    help="choose the chunk size with the autotuner (candidates 16, 32, 64, 128) "
                         "before timing; the default keeps the workload's chunk of 64")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the plain unfused form (the speed-up denominator)")
    ap.add_argument("--solver", type=int, default=0, metavar="ITERS",
                    help="instead of the gradient step, time ITERS conjugate-gradient "
                         "iterations (holo_cg) from u and the back-propagated reference probe "
                         "and print their own JSON line")
    ap.add_argument("--batch2d", action="store_true",
                    help="time only the batched single-angle workload (96 instances) and print "
                         "its own JSON line")
    ap.add_argument("--no-batch2d", action="store_true",
                    help="leave the batched single-angle workload out of the default line")
    ap.add_argument("--no-fourier", action="store_true",
                    help="leave the Fourier-slice projector's gradient out of the default line")
    ap.add_argument("--cpu-baseline-child", metavar="DIR", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_baseline_child)
        return
    if args.gpus != 1:
        print("bench.py measures one MI355X: the path runs on a single GPU "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2407_20304_amd import holo, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    holo.lib()  # fails loudly if the HIP library is missing
    if args.batch2d:
        res = batch2d_bench()
        res.update({"metric": "batched single-angle gradient calls/s", "value": res["calls_per_s"],
                    "unit": "calls/s", "n_gpus": 1, "higher_is_better": True, "dtype": "c64",
                    "data": "synthetic"})
        print(json.dumps(res), flush=True)
        return
    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS[args.workload]
    H, W, N, nd = wl.H, wl.W, wl.n_angles, len(wl.mag_rel)
    sd = lambda role: synth.seed_of(wl.config, role)

    log("inputs: %s (volume %dx%dx%d, %d angles, %d planes, detector %dx%d)"
        % (wl.name, H, W, W, N, nd, H, W))
    u = synth.ellipsoid_volume(W, H, sd(4), device=dev)
    q_np = synth.probe(H, W, sd(5))
    q = torch.from_numpy(q_np).to(dev)
    amp = synth.synthetic_amplitudes(N, nd, H, W, sd(9), device=dev)
    amp_ref = synth.synthetic_amplitudes(1, 1, H, W, sd(9) + 500, device=dev)[0, 0].contiguous()
    torch.cuda.synchronize()
    log("inputs ready")

    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read + 1 GiB written")

    plan = holo.Plan.for_workload(wl)
    if args.overlap is not None:
        plan.set_tile("overlap", args.overlap)
    if args.fwd_bins is not None:
        plan.set_tile("fwd_bins", args.fwd_bins)
    if args.col_tile is not None:
        plan.set_tile("col_tile", args.col_tile)
    tuned = None
    if args.tune:
        best, times = plan.autotune(u, q, amp, amp_ref, candidates=(16, 32, 64, 128))
        tuned = {"chunk": best, "ms": times}
        log("autotune: chunk %d (%s)" % (best, times))
    if args.solver > 0:
        solver_bench(args, wl, plan, u, amp, amp_ref)
        return
    ws = plan.workspace(dev)
    F = torch.empty((1,), dtype=torch.float64, device=dev)
    g_u = torch.empty_like(u)
    g_q = torch.empty_like(q)
    log("workspace %.1f GiB" % (plan.workspace_bytes / 2 ** 30))

    for i in range(args.warmup):
        plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=g_u, g_q=g_q)
        torch.cuda.synchronize()
        log("warmup %d done" % i)

    plan.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=g_u, g_q=g_q)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.timing(False)
    kt = plan.kernel_times()
    log("timed %d steps: %.3f s" % (args.steps, elapsed))
    Fv = F.item()
    if not math.isfinite(Fv):
        print("objective is not finite", file=sys.stderr)
        sys.exit(1)

    K = args.steps
    lerps = float(N) * W * W * H * K
    kernels = {}
    for name, (ms, n) in kt.items():
        if n == 0:
            continue
        ent = {"ms_per_step": ms / K, "launches_per_step": n / K, "avg_launch_ms": ms / n}
        if name in ("radon_fwd", "radon_adj"):
            tf = lerps * FLOP_PER_LERP / (ms * 1e-3) / 1e12
            ent.update({"achieved": tf, "unit": "TFLOP/s", "frac": tf / PEAK_FP32_VALU_TFLOPS,
                        "traffic_per_launch": traffic_bytes("k_" + name, wl.name)})
        kernels[name] = ent
    frame_ms = sum(kt[c][0] for c in ("pass_a", "pass_b", "pass_c", "pass_d"))
    frame_gbs = frame_bytes_model(wl, K) / (frame_ms * 1e-3) / 1e9 if frame_ms > 0 else None
    dom = max(("radon_fwd", "radon_adj"), key=lambda c: kt[c][0])
    dms, dn = kt[dom]
    per_launch_flop = lerps * FLOP_PER_LERP / dn
    achieved = per_launch_flop / (dms / dn * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_" + dom, "achieved": achieved,
                "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic_bytes("k_" + dom, wl.name),
                "per_launch_flop": per_launch_flop, "avg_launch_ms": dms / dn}

    result = {
        "metric": METRIC,
        "value": K / elapsed,
        "unit": "gradient evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": wl.name, "volume": [H, W, W], "n_angles": N, "chunk": plan.chunk,
                   "overlap": plan.get_tile("overlap"),
                   "fwd_bins": plan.get_tile("fwd_bins"),
                   "col_tile": plan.get_tile("col_tile"),
                   "n_dist": nd, "detector": [H, W], "parallelism": "single GPU"},
        "objective": Fv,
        "frame_stage_GBps": frame_gbs,
        "frame_stage_hbm_frac": None if frame_gbs is None else frame_gbs / PEAK_HBM_GBS,
        "kernels": kernels,
        "roofline": roofline,
    }
    if tuned is not None:
        result["autotune"] = tuned
    if not args.no_plain:
        result["plain"] = plain_bench(wl, u, q, amp, amp_ref, F, g_u, g_q, K / elapsed)
        result["vs_plain"] = result["plain"]["speedup"]
    if not args.no_fourier and W <= 1024:
        log("Fourier-slice projector")
        plan.close()
        del ws, plan
        torch.cuda.empty_cache()
        result["fourier_slice"] = fourier_bench(wl, u, q, amp, amp_ref, K, K / elapsed, Fv)
    if not args.no_batch2d:
        log("batched single-angle workload")
        result["batch2d"] = batch2d_bench()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        result["cpu_baseline"] = cpu_baseline(wl, u, q_np, amp, amp_ref.cpu().numpy(),
                                              args.cpu_slab)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
