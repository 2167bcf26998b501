"""Benchmark of the extended-LBGK hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): D3Q27 decaying
homogeneous isotropic turbulence, 256^3 periodic, cubic lattice, T = 0.5,
omega = 1.892885 (Re_lambda = 72 for the k0 = 4 spectrum), u_rms = 0.05,
rho = 1, seeded solenoidal field with E(k) ~ k^4 exp(-2 (k/k0)^2). One step is
one fused stream-and-collide launch over the whole lattice; FP64 kinetic
energy / enstrophy reductions run every 50 steps inside the timed region,
as in the workload. Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS (FP32 deviation storage) as `value`, the FP16 and
BF16 deviation-storage runs of the same workload beside it (whole-job and
kernel-time ratios), the roofline of the step kernel (algorithmic bytes 2 Q s
per node, measured with HIP events on the launch stream) with the achievable
ceiling measured by the bandwidth probe, the channel and D2Q9 workloads, the
served mixed stream at its own rate (saturated) and at half of it (under
capacity), and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "D3Q27 MLUPS & % HBM roofline, FP32 vs FP16-store; served solves/s + p99"
N_HIT = 256
OMEGA_HIT = 1.892885
T_HIT = 0.5
DIAG_EVERY = 50
# Channel workload (Sec. 3.5 at Re_tau = 180): 384 x 192 x 192 on the lattice
# stretched to lambda = (2, 1, 1), half-width H = 96 rows, T = 0.5; omega from
# the friction-velocity estimate, the force g = Re_tau^2 nu^2 / H^3.
CHANNEL_N = (384, 192, 192)
CHANNEL_LAM = (2.0, 1.0, 1.0)
CHANNEL_H = 96
CHANNEL_RE_TAU = 180.0
CHANNEL_T = 0.5
CHANNEL_OMEGA = 1.976785
PMC_FILE = os.path.join(ROOT, "profiles", "step_d3q27_f32_hit256_pmc.txt")
STEP_SOURCE = os.path.join(ROOT, "paper_2101_04550_amd", "csrc", "elbm_step.hip")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storages", default="f32,f16,bf16")
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--n", type=int, default=N_HIT, help="cube edge (default 256)")
    ap.add_argument("--kernel-reps", type=int, default=200, help="step launches timed for the roofline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the served mixed stream (0: skip the serving leg)")
    ap.add_argument("--channel-only", action="store_true",
                    help="only the 384x192x192 channel leg (FP32 and FP16), one JSON line: for per-kernel profiles")
    ap.add_argument("--no-ceiling", action="store_true", help="omit the bandwidth-ceiling probe")
    ap.add_argument("--ceiling-only", action="store_true",
                    help="only the bandwidth-ceiling probe, one JSON line: for its kernel profile")
    ap.add_argument("--mrt-only", action="store_true",
                    help="only the multi-relaxation-time collision against LBGK (D3Q27 256^3, D2Q9 4096^2), "
                         "one JSON line")
    ap.add_argument("--hit-only", action="store_true",
                    help="only the 256^3 turbulence legs (no D2Q9 or serving leg): for per-kernel profiles")
    return ap.parse_args()


def step_source_hash():
    with open(STEP_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_pmc_traffic():
    """HBM bytes per step launch from the committed rocprofv3 counter summary,
    scaled by the copy-kernel calibration; None if absent or stale."""
    if not os.path.exists(PMC_FILE):
        return None
    kv = {}
    for line in open(PMC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("step_source_sha256") != step_source_hash():
            return None
        fetch = float(kv["step_fetch_kib_per_dispatch"]) * 1024 / float(kv["copy_fetch_factor"])
        write = float(kv["step_write_kib_per_dispatch"]) * 1024 / float(kv["copy_write_factor"])
        return fetch + write
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def calibrate_copy():
    import torch

    n = 1 << 29  # 2 GiB of fp32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 4, "bytes_written": n * 4, "launches": 5}))


def run_gpu(storage, fld, steps, warmup, kernel_reps):
    import torch

    from paper_2101_04550_amd import elbm as E

    n = fld.n
    N = math.prod(n)
    # Both lattices are set up first, so that no host work (initial fields,
    # uploads) separates the two timed parts: the GPU's clocks drop within a
    # fraction of a second of idling and take ~30-60 launches (~20 ms) to come
    # back, which would put a short whole-job window into the ramp (the
    # 16-bit kernels, more arithmetic-bound, run 5-9% slower during it).
    p2 = E.make_params(n, T=T_HIT, omega=OMEGA_HIT, storage=storage)
    kl = E.Lattice(p2)
    kl.init(fld.rho, fld.u)
    params = E.make_params(n, T=T_HIT, omega=OMEGA_HIT, storage=storage, diag_every=DIAG_EVERY,
                           diag_capacity=max(1, (steps + warmup) // DIAG_EVERY + 1))
    lat = E.Lattice(params)
    lat.init(fld.rho, fld.u)
    info = lat.kernel_info()
    stream = lat.stream
    # step-kernel duration: diagnostics off, events on the launch stream around
    # kernel_reps back-to-back step launches, after 60 untimed ones (past the
    # clock ramp that follows the set-up)
    kl.step(60)
    kl.sync()
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(kl.stream)
    kl.step(kernel_reps)
    k1.record(kl.stream)
    # whole-job timed region: W warm-up steps, then exactly K steps (with the
    # FP64 diagnostics of every 50th step), bracketed by synchronisations
    lat.step(warmup)
    lat.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    t1.synchronize()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    kms = k0.elapsed_time(k1) / kernel_reps
    d = kl.diag()
    kl.close()
    del kl
    hist = lat.diag_history()
    timed = [h for h in hist if warmup < h["step"] <= warmup + steps]
    lat.close()
    del lat
    torch.cuda.empty_cache()
    es = 4 if storage == "f32" else 2
    alg_bytes = 2 * 27 * es * N
    return {
        "storage": storage,
        "mlups": N * steps / (ms * 1e-3) / 1e6,
        "ms_per_step": ms / steps,
        "kernel_ms": kms,
        "kernel_gbs": alg_bytes / (kms * 1e-3) / 1e9,
        "alg_bytes_per_launch": alg_bytes,
        "diag_samples_timed": len(timed),
        "ke_first": hist[0]["ke"] if hist else None,
        "ke_last": hist[-1]["ke"] if hist else None,
        "enstrophy_last": hist[-1]["enstrophy"] if hist else None,
        "final_min_rho": d["min_rho"],
        "kernel": info,
    }


def serving_leg(nreq, rate):
    """Continuous batching of the seeded mixed stream: Poisson arrivals at
    `rate` req/s, 10% D3Q27 turbulence boxes (64^3..192^3), the rest D2Q9 shear
    waves and double shear layers (64^2..1024^2), cubic or stretched, T in
    {1/3, 1/2}, 200..5000 steps, FP32 / FP16 storage. Latency = completion -
    arrival; offered_glups = the stream's node updates over its arrival
    window (above the sustained rate the queue grows and latency measures the
    backlog)."""
    import torch

    from paper_2101_04550_amd import serving as SV

    reqs = SV.attach_fields(SV.make_stream(nreq, rate=rate, share_3d=0.1))
    window = reqs[-1].arrival
    offered = sum(r.cells * r.steps for r in reqs)
    srv = SV.Server(64 * 2 ** 30, max_slots=64, quantum=100, use_graph=True)
    res = srv.run(reqs)
    out = SV.summarize(res, srv.makespan)
    out.update({"arrival_rate_per_s": rate, "share_3d": 0.1, "quantum_steps": 100, "rounds": srv.rounds,
                "peak_slots": srv.peak_slots, "pool_gb": 64, "arrival_window_s": window,
                "offered_glups": offered / window / 1e9})
    srv.close()
    torch.cuda.empty_cache()
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}


def ceiling_leg(n=N_HIT, reps=20):
    """Achievable bandwidth of the step's access pattern on this device: the
    population traffic of one D3Q27 step (27 pulled loads and 27 nontemporal
    stores per node, plane slabs) without arithmetic (libelbm_probe.so), at
    the step kernels' occupancies and at full occupancy, FP32 and FP16; and a
    plain device copy (torch) of 2 GiB."""
    import ctypes as C

    import torch

    from paper_2101_04550_amd import elbm as E  # noqa: F401  (same HIP runtime as torch)

    lib = C.CDLL(os.path.join(ROOT, "paper_2101_04550_amd", "libelbm_probe.so"))
    lib.elbm_probe_bytes.argtypes = [C.c_int32] * 4 + [C.POINTER(C.c_size_t)]
    lib.elbm_probe_stream.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int32] * 8 + [C.c_void_p, C.POINTER(C.c_float)]
    lib.elbm_probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_void_p, C.POINTER(C.c_float)]
    out = {}
    st = torch.cuda.current_stream()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    plane_blocks = (n * n + 511) // 512
    for es, name in ((4, "f32"), (2, "f16")):
        nb = C.c_size_t(0)
        assert lib.elbm_probe_bytes(es, n, n, n, C.byref(nb)) == 0
        a = torch.zeros(nb.value, dtype=torch.uint8, device="cuda")
        b = torch.zeros_like(a)
        res = {}
        # blocks of 512 threads per CU: 1 (the FP32 step kernel's 8 waves), 2
        # (the FP16 staged kernel's 16 waves), 4 (full occupancy of the probe)
        for bpc, lds in ((1, 96 * 1024), (2, 64 * 1024), (4, 0)):
            chunk = max(1, n * plane_blocks // (cus * bpc))
            ms = C.c_float(0)
            rc = lib.elbm_probe_stream(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), es, n, n, n, chunk, 1,
                                       lds, reps, C.c_void_p(st.cuda_stream), C.byref(ms))
            assert rc == 0, rc
            res[f"{bpc * 8}_waves_per_cu"] = round(2 * 27 * es * n ** 3 / (ms.value * 1e-3) / 1e9, 1)
        out[name] = res
        del a, b
        torch.cuda.empty_cache()
    x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    res = {}
    for per_cu in (2, 4, 8):
        for unroll in (1, 2, 4):
            ms = C.c_float(0)
            rc = lib.elbm_probe_copy(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel() * 4,
                                     cus * per_cu, unroll, reps, C.c_void_p(st.cuda_stream), C.byref(ms))
            assert rc == 0, rc
            res[f"{per_cu * 4}_waves_per_cu_x{unroll}"] = round(2 * x.numel() * 4 / (ms.value * 1e-3) / 1e9, 1)
    out["copy16"] = res
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    out["torch_copy_gbs"] = round(2 * x.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    out["best_gbs"] = max([v for k in ("f32", "f16", "copy16") for v in out[k].values()] + [out["torch_copy_gbs"]])
    out["unit"] = "GB/s (read + written)"
    return out


def d2q9_leg(n=1024, steps=10000):
    """D2Q9 double shear layer n^2 (T = 0.5, Re = 3e4: omega = 1.973061),
    10000 steps (t* = 0.98) in FP32 and FP16 storage, with the LBGK collision
    and with the multi-relaxation-time one (omega_bulk = 1, omega_ghost =
    1.5): at these parameters LBGK is linearly unstable about the layer's
    stream and diverges within the run, the MRT collision runs it (same
    kernel, a runtime branch). At 1024^2 both buffers (75 MB FP32) fit the
    256 MB last-level cache, so the rate is not an HBM figure."""
    import torch

    import inputs as I
    from paper_2101_04550_amd import elbm as E

    fld = I.double_shear_layer((n, n))
    out = {}
    for st in ("f32", "f16"):
        for tag, kw in (("", {}), ("_mrt", dict(omega_bulk=1.0, omega_ghost=1.5))):
            lat = E.Lattice(E.make_params((n, n), T=0.5, omega=1.973061, storage=st, **kw))
            lat.init(fld.rho, fld.u)
            lat.step(20)
            lat.sync()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(lat.stream)
            lat.step(steps - 20)
            b.record(lat.stream)
            b.synchronize()
            ms = a.elapsed_time(b) / (steps - 20)
            es = 4 if st == "f32" else 2
            d = lat.diag(check=False)
            finite = bool(d["nan_count"] == 0 and math.isfinite(d["ke"]))
            out[st + tag] = {"mlups": round(n * n / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 5),
                             "alg_gbs": round(2 * 9 * es * n * n / (ms * 1e-3) / 1e9, 1),
                             "finite_at_end": finite,
                             "ke_end": d["ke"] if finite else None,
                             "enstrophy_end": d["enstrophy"] if finite else None}
            lat.close()
    torch.cuda.empty_cache()
    out["note"] = (f"D2Q9 {n}^2 double shear layer, {steps} steps; cache-resident (not an HBM roofline); "
                   "LBGK at T = 0.5, Re = 3e4 is linearly unstable about the layer's stream (diverges), "
                   "the MRT collision (omega_bulk 1, omega_ghost 1.5) runs it")
    return out


def channel_force():
    """Body force of the channel workload, g = Re_tau^2 nu^2 / H^3 (Sec. 3.5),
    with nu = (1/omega - 1/2) T (Sec. 2.1, eq. nu)."""
    nu = (1 / CHANNEL_OMEGA - 0.5) * CHANNEL_T
    return CHANNEL_RE_TAU ** 2 * nu ** 2 / CHANNEL_H ** 3


def channel_leg(steps=300):
    """D3Q27 channel on the stretched lattice (dy/dx = 0.5): 384 x 192 x 192,
    bounce-back walls in y, body force for Re_tau = 180, T = 0.5,
    omega = 1.976785; FP32 and FP16 storage, step rate after 20 warm-up steps
    (the workload's 5000-step run is the same kernel)."""
    import torch

    import inputs as I
    from paper_2101_04550_amd import elbm as E

    n, lam, omega = CHANNEL_N, CHANNEL_LAM, CHANNEL_OMEGA
    g = channel_force()
    fld = I.channel_field(n, lam)
    N = math.prod(n)
    out = {}
    for st in ("f32", "f16"):
        lat = E.Lattice(E.make_params(n, lam=lam, T=CHANNEL_T, omega=omega, walls=(False, True, False),
                                      force=(g, 0.0, 0.0), storage=st))
        lat.init(fld.rho, fld.u)
        info = lat.kernel_info()
        lat.step(20)
        lat.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(lat.stream)
        lat.step(steps)
        b.record(lat.stream)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        es = 4 if st == "f32" else 2
        out[st] = {"mlups": round(N / (ms * 1e-3) / 1e6, 1), "kernel_ms": round(ms, 5),
                   "alg_gbs": round(2 * 27 * es * N / (ms * 1e-3) / 1e9, 1), "kernel": info["kernel"]}
        lat.close()
    torch.cuda.empty_cache()
    out["note"] = "D3Q27 channel 384x192x192, lambda = (2, 1, 1), walls in y, Re_tau = 180 force"
    return out


def mrt_leg(steps=200):
    """Step time of the multi-relaxation-time collision (omega_bulk = 1.2,
    omega_ghost = 1.0) beside LBGK on the same lattice: D3Q27 256^3
    turbulence (T = 0.5) in FP32 / FP16 / BF16 and the D2Q9 4096^2 double
    shear layer (T = 0.5, omega = 1.9) in FP32 / FP16; HIP events over
    `steps` steps after 30 warm-up steps, no sample steps."""
    import torch

    import inputs as I
    from paper_2101_04550_amd import elbm as E

    def one(params, fld):
        lat = E.Lattice(params)
        lat.init(fld.rho, fld.u)
        lat.step(30)
        lat.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(lat.stream)
        lat.step(steps)
        b.record(lat.stream)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        kern = lat.kernel_info()["kernel"]
        N = lat.N
        lat.close()
        return {"ms": round(ms, 5), "mlups": round(N / (ms * 1e-3) / 1e6, 1), "kernel": kern}

    rates = dict(omega_bulk=1.2, omega_ghost=1.0)
    out = {}
    fld = I.hit_field(N_HIT, k0=4.0, urms=0.05)
    for st in ("f32", "f16", "bf16"):
        base = dict(T=0.5, omega=OMEGA_HIT, storage=st)
        out[f"d3q27_{N_HIT}_{st}"] = {
            "lbgk": one(E.make_params((N_HIT,) * 3, **base), fld),
            "mrt": one(E.make_params((N_HIT,) * 3, **base, **rates), fld)}
    del fld
    torch.cuda.empty_cache()
    n2 = (4096, 4096)
    fld = I.double_shear_layer(n2)
    for st in ("f32", "f16"):
        base = dict(T=0.5, omega=1.9, storage=st)
        out[f"d2q9_4096_{st}"] = {"lbgk": one(E.make_params(n2, **base), fld),
                                  "mrt": one(E.make_params(n2, **base, **rates), fld)}
    torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds_budget=20.0):
    """The FP64 NumPy oracle (untuned) on a bounded sample of the same workload:
    a 96^3 box of the same spectrum (k0 = 4), timed over whole steps, on one
    thread (the BLAS and OpenMP pools NumPy may use are capped to one thread
    for the timed run)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import inputs as I
    import oracle as O

    n = 96
    fld = I.hit_field(n, k0=4.0, urms=0.05)
    p = O.Params(n=(n, n, n), T=T_HIT, omega=OMEGA_HIT)
    f = O.init_state(fld.rho, fld.u, p)
    with threadpool_limits(limits=1):
        pools = sorted({(pl["internal_api"], pl["num_threads"]) for pl in threadpool_info()})
        f = O.step(f, p)  # warm caches / allocator
        steps = 0
        t = time.perf_counter()
        while True:
            f = O.step(f, p)
            steps += 1
            if time.perf_counter() - t > seconds_budget or steps >= 200:
                break
        dt = time.perf_counter() - t
    assert np.isfinite(f).all()
    cpu = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": n ** 3 * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"D3Q27 HIT {n}^3 (k0=4, T=0.5, omega={OMEGA_HIT}), {steps} FP64 NumPy steps in "
                  f"{dt:.1f} s on one core of {cpu} ({os.cpu_count()} logical CPUs visible)",
        "thread_pools": [f"{api}:{k}" for api, k in pools],
    }


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(a lattice runs on one GPU; sharding it across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.channel_only:
        print(json.dumps({"channel": channel_leg()}), flush=True)
        return
    if args.ceiling_only:
        print(json.dumps({"ceiling": ceiling_leg()}), flush=True)
        return
    if args.mrt_only:
        print(json.dumps({"mrt": mrt_leg()}), flush=True)
        return
    import torch

    import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fld = I.hit_field(args.n, k0=4.0, urms=0.05)
    runs = {}
    for s in [x for x in args.storages.split(",") if x]:
        runs[s] = run_gpu(s, fld, args.steps, args.warmup, args.kernel_reps)
        print(f"# {s}: {runs[s]['mlups']:.1f} MLUPS, step kernel {runs[s]['kernel_ms']:.4f} ms "
              f"= {runs[s]['kernel_gbs']:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    main_run = runs.get("f32") or next(iter(runs.values()))
    N = args.n ** 3
    traffic = read_pmc_traffic() if (args.n == N_HIT and main_run["storage"] == "f32") else None
    out = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_run["storage"],
        "data": "synthetic",
        "config": {
            "workload": f"D3Q27 decaying HIT {args.n}^3 periodic, cubic lattice, T=0.5, omega={OMEGA_HIT}, "
                        f"u_rms=0.05, k0=4; {main_run['storage'].upper()} deviation storage; FP64 KE/enstrophy "
                        f"every {DIAG_EVERY} steps ({main_run['diag_samples_timed']} in the timed window)",
            "lattice": "D3Q27",
            "cells": N,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(main_run["kernel_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_run["kernel_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / (main_run["kernel_ms"] * 1e-3) / 1e9, 1),
            "kernel": "step_kernel<D3Q27, f32, periodic, no force>",
            "kernel_ms": round(main_run["kernel_ms"], 5),
            "alg_bytes_per_launch": main_run["alg_bytes_per_launch"],
        },
        "storage_variants": {
            s: {"mlups": round(r["mlups"], 1), "kernel_ms": round(r["kernel_ms"], 5),
                "kernel_gbs": round(r["kernel_gbs"], 1),
                "vs_f32": round(r["mlups"] / main_run["mlups"], 3),
                "vs_f32_whole_job": round(r["mlups"] / main_run["mlups"], 3),
                "vs_f32_kernel": round(main_run["kernel_ms"] / r["kernel_ms"], 3),
                "diag_samples_timed": r["diag_samples_timed"],
                "kernel": "step_kernel_lds (LDS staged)" if r["kernel"]["kernel"] == "staged"
                else "step_kernel (register pull)",
                "block_threads": r["kernel"]["block_threads"], "tile": list(r["kernel"]["tile"])}
            for s, r in runs.items()
        },
        "diagnostics": {s: {"ke_first": r["ke_first"], "ke_last": r["ke_last"],
                            "enstrophy_last": r["enstrophy_last"], "min_rho": r["final_min_rho"]}
                        for s, r in runs.items()},
    }
    if args.n == N_HIT and not args.hit_only:
        out["d2q9"] = d2q9_leg()
        out["channel"] = channel_leg()
        out["mrt"] = mrt_leg()
    if args.n == N_HIT and not args.no_ceiling:
        out["ceiling"] = ceiling_leg()
        out["roofline"]["ceiling_gbs"] = out["ceiling"]["best_gbs"]
        out["roofline"]["frac_of_ceiling"] = round(out["roofline"]["achieved"] / out["ceiling"]["best_gbs"], 4)
        print(f"# ceiling: {out['ceiling']}", file=sys.stderr, flush=True)
    if args.serve_requests > 0 and args.n == N_HIT and not args.hit_only:
        # the stream's own rate (50 req/s: offered above what the GPU sustains,
        # latency includes the backlog), then half of it (under capacity)
        out["serving"] = {}
        for rate in (50.0, 25.0):
            out["serving"][f"rate_{int(rate)}"] = serving_leg(args.serve_requests, rate)
        cap = out["serving"]["rate_50"]["sustained_glups"]
        for key, sv in out["serving"].items():
            sv["regime"] = "under capacity" if sv["offered_glups"] < 0.95 * cap else "saturated"
            print(f"# serving {key} ({sv['regime']}): {sv['solves_per_s']:.1f} solves/s, "
                  f"p50 {sv['p50_latency_s']:.3f} s, p99 {sv['p99_latency_s']:.3f} s", file=sys.stderr, flush=True)
    if not args.skip_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
