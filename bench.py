"""Benchmark of the LW-ACM time step on one MI355X.

Workload: D3Q19 Taylor-Green vortex on a 256^3 periodic grid (u0 = 0.02,
omega = 1.7), synthetic initial field, state resident in HBM.  A timed step
is one full forward step (gather, link terms, post-combine, normalisation,
store, fused FP64 mass/energy reduction); the library runs FP32 steps two
per launch (the intermediate state stays on chip).  Reported beside it: the
single-step kernel, the same step with FP16-deviation storage, the reverse
(adjoint) step and the checkpointed forward+reverse cost, the rooflines of
the forward kernel (HBM at 32 bytes per lattice update, and VALU issue),
and the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS D3Q19 256^3 FP32 (vs FP16-store); adjoint/forward step time ratio"
HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 FP32 instruction per 4 cycles, 2.4 GHz
VALU_WAVE_INSTS_PER_S = 1024 * 2.4e9 / 4
FP32_PEAK_TFLOPS = 157.3           # packed FP32 FMA (published vector peak)
FP32_UNPACKED_TFLOPS = 78.6        # one FP32 FMA per lane per cycle (the kernels use no packed FP32)
# FP32 operations of one lattice update in the tile kernels (Eqs. ACM2.0b as
# implemented, mass/energy sums included): 47 FMA, 40 add/sub, 22 mul, 1 rcp
FLOPS_PER_UPDATE = 2 * 47 + 40 + 22 + 1


def _measured(kernel: str, key: str = "hbm_bytes_per_launch"):
    """A counter-derived figure of `kernel` (HBM bytes per launch from its
    FETCH_SIZE/WRITE_SIZE runs scaled by the copy-kernel calibration, or its
    VALU instructions per launch), or None when the kernel's sources changed
    since the counters were taken."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_1111_2142_amd")
    try:
        rec = json.load(open(os.path.join(pkg, "measured_traffic.json")))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    return rec.get(key) if h.hexdigest() == rec["sources_sha256"] else None


def _measured_traffic(kernel: str):
    return _measured(kernel, "hbm_bytes_per_launch")


def _events_time(fn, n, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    fn(n)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3  # seconds


def _stream_reference(dev):
    """GB/s of bench_stream_ref.hip's copy (bytes read + written), read and
    write of 1 GiB, each under the cache policies 0 (default), 2 (nt), 16
    (sc1), 18 (nt, sc1) and two grid sizes; the best of each kind beside
    torch's own device copy."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "bench_stream_ref.so"))
    lib.stream_ref_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_uint, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_float)]
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    out = {}
    for kind, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes), (2, "write", nbytes)):
        for pol in (0, 2, 16, 18):
            for grid in (2048, 8192):
                ms = ctypes.c_float(0.0)
                rc = lib.stream_ref_run(kind, pol, dst.data_ptr(), src.data_ptr(), nbytes, grid,
                                        20, ctypes.byref(ms))
                if rc != 0:
                    raise RuntimeError(f"stream_ref_run({kind}, {pol}, {grid}) = {rc}")
                out[f"{name}_p{pol}_g{grid}"] = round(moved / (ms.value * 1e-3) / 1e9, 1)
    for _ in range(3):
        dst.copy_(src)
    t = _events_time(lambda k: [dst.copy_(src) for _ in range(k)], 20,
                     torch.cuda.current_stream(dev))
    out["torch_copy"] = round(2 * nbytes * 20 / t / 1e9, 1)
    for name in ("copy", "read", "write"):
        out[f"best_{name}"] = max(v for k, v in out.items() if k.startswith(name + "_"))
    print(f"[bench] streaming reference GB/s: copy {out['best_copy']}, read {out['best_read']}, "
          f"write {out['best_write']}, torch copy {out['torch_copy']}", file=sys.stderr, flush=True)
    return out


def _cavity_leg(args, L, wl, dev, stream):
    """The 192^3 lid-driven cavity: walls on every face, the lid moving.  The
    masked one-step kernel moves 36 B per node: the state read and written
    (2 x 16 B) and the node's 32-bit set of solid upstream links."""
    import torch
    c4 = wl.CAVITY_192
    m4 = torch.as_tensor(wl.cavity_mask(c4.nx), device=dev)
    s4 = L.Solver(L.LWACM_D3Q19, c4.nx, c4.ny, c4.nz, c4.omega, mask=m4,
                  wall_u=[list(r) for r in wl.wall_table(c4.lid)], device=dev)
    s4.set_state(torch.zeros((c4.nz, c4.ny, c4.nx), device=dev),
                 torch.zeros((3, c4.nz, c4.ny, c4.nx), device=dev))
    s4.step(args.warmup)
    dt4 = _events_time(s4.step, args.steps, stream)
    # momentum-exchange force and torque on the walls at rest (mask id 1;
    # lwacm_wall_force): one pass over the grid and a fixed-order FP64 sum,
    # host-synchronised
    import time
    c = (c4.nx - 1) / 2.0
    s4.wall_force(1, (c, c, c))
    t0 = time.perf_counter()
    for _ in range(10):
        f_w, t_w = s4.wall_force(1, (c, c, c))
    ms_force = (time.perf_counter() - t0) / 10 * 1e3
    s4.close()
    fluid4 = (c4.nx - 2) * (c4.ny - 2) * (c4.nz - 2)
    ms4 = dt4 / args.steps * 1e3
    print(f"[bench] cavity 192^3: {ms4:.4f} ms/step; wall force {ms_force:.3f} ms per call",
          file=sys.stderr, flush=True)
    return {"value": round(fluid4 * args.steps / dt4 / 1e6, 1), "unit": "MLUPS (fluid nodes)",
            "ms_per_step": round(ms4, 5), "omega": c4.omega, "lid": list(c4.lid),
            "achieved_GBs": round(36.0 * c4.nx * c4.ny * c4.nz / (ms4 * 1e-3) / 1e9, 1),
            "basis": "36 B per node: state in and out, 32-bit solid-link set",
            "wall_force_ms": round(ms_force, 4),
            "walls_at_rest_force": [round(v, 8) for v in f_w],
            "walls_at_rest_torque": [round(v, 8) for v in t_w],
            "kernel": "k_fwd_march2<64,true>",
            "traffic": _measured_traffic("k_fwd_march2<64,true>")}


def _qbb_leg(args, L, wl, dev, stream):
    """The 192^3 lid-driven cavity with interpolated bounce-back: every wall
    cuts its links at q = 0.3 (d_q of lwacm_init).  Each step is the wall
    correction over the fluid nodes next to a wall (k_wall_correction: the
    whole wall term of each) and the masked single-step tile kernel, which
    adds it in place of its own bounce-back sums."""
    import torch
    c4 = wl.CAVITY_192
    m4 = torch.as_tensor(wl.cavity_mask(c4.nx), device=dev)
    qd = torch.full((19, c4.nz, c4.ny, c4.nx), 0.3, dtype=torch.float32, device=dev)
    s8 = L.Solver(L.LWACM_D3Q19, c4.nx, c4.ny, c4.nz, c4.omega, mask=m4,
                  wall_u=[list(r) for r in wl.wall_table(c4.lid)], device=dev, qd=qd)
    s8.set_state(torch.zeros((c4.nz, c4.ny, c4.nx), device=dev),
                 torch.zeros((3, c4.nz, c4.ny, c4.nx), device=dev))
    s8.step(args.warmup)
    dt8 = _events_time(s8.step, args.steps, stream)
    s8.close()
    del qd, m4
    torch.cuda.empty_cache()
    fluid = (c4.nx - 2) * (c4.ny - 2) * (c4.nz - 2)
    ms8 = dt8 / args.steps * 1e3
    print(f"[bench] cavity 192^3 interpolated walls: {ms8:.4f} ms/step", file=sys.stderr,
          flush=True)
    return {"value": round(fluid * args.steps / dt8 / 1e6, 1), "unit": "MLUPS (fluid nodes)",
            "ms_per_step": round(ms8, 5), "q": 0.3,
            "achieved_GBs": round(33.0 * c4.nx * c4.ny * c4.nz / (ms8 * 1e-3) / 1e9, 1),
            "kernel": "k_fwd_march_rolled<float,64,false,true,false,0,true,false> + k_wall_correction<float>",
            "traffic": _measured_traffic("k_fwd_march_rolled<float,64,false,true,false,0,true,false>"),
            "basis": "33 B per node (state in and out, uint8 mask), the figure of the halfway "
                     "cavity; the wall correction reads the state, q and the second node of "
                     "the fluid nodes next to a wall and writes one float4 for each"}


def _split_leg(args, L, wl, dev, stream, drho_t, u_t, n):
    """The 256^3 Taylor-Green step with a separate omega_p for the density
    (nu_p = 10 nu): the single-step tile kernel with its eight extra LDS
    partials per node."""
    cfg = wl.TGV3D_256
    nu = (1.0 / cfg.omega - 0.5) / 3.0
    s6 = L.Solver(L.LWACM_D3Q19, n, n, n, cfg.omega, device=dev,
                  omega_p=wl.omega_for_viscosity(10.0 * nu))
    s6.set_state(drho_t, u_t)
    s6.step(args.warmup)
    dt6 = _events_time(s6.step, args.steps, stream)
    s6.close()
    ms6 = dt6 / args.steps * 1e3
    nodes = n ** 3
    print(f"[bench] omega_p split {n}^3: {ms6:.4f} ms/step", file=sys.stderr, flush=True)
    kname = "k_fwd_march_rolled<float,128,false,false,true,0,false,false>"
    return {"value": round(nodes * args.steps / dt6 / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms6, 5), "nu_p_over_nu": 10.0,
            "achieved_GBs": round(32.0 * nodes / (ms6 * 1e-3) / 1e9, 1),
            "frac": round(32.0 * nodes / (ms6 * 1e-3) / 8.0e12, 4),
            "kernel": kname if n == 256 else None,
            "traffic": _measured_traffic(kname) if n == 256 else None,
            "basis": "32 B per update (state read and written); one step per launch: the "
                     "single-step tile kernel with eight more LDS partials per node"}


def _field_leg(args, L, wl, dev, stream, drho_t, u_t, n):
    """The 256^3 Taylor-Green step with a body acceleration given node by node
    (lwacm_set_force_field): the single-step tile kernel, which also reads the
    three acceleration fields (44 B per update)."""
    import torch
    cfg = wl.TGV3D_256
    s7 = L.Solver(L.LWACM_D3Q19, n, n, n, cfg.omega, device=dev)
    s7.set_state(drho_t, u_t)
    g = 1e-7 * u_t.clone()  # any smooth field of the grid's shape
    s7.set_force_field(g)
    s7.step(args.warmup)
    dt7 = _events_time(s7.step, args.steps, stream)
    s7.close()
    del g
    torch.cuda.empty_cache()
    ms7 = dt7 / args.steps * 1e3
    nodes = n ** 3
    print(f"[bench] force field {n}^3: {ms7:.4f} ms/step", file=sys.stderr, flush=True)
    return {"value": round(nodes * args.steps / dt7 / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms7, 5),
            "achieved_GBs": round(44.0 * nodes / (ms7 * 1e-3) / 1e9, 1),
            "frac": round(44.0 * nodes / (ms7 * 1e-3) / 8.0e12, 4),
            "kernel": "k_fwd_march_rolled<float,128,false,false,false,2,false,false>" if n == 256 else None,
            "traffic": _measured_traffic("k_fwd_march_rolled<float,128,false,false,false,2,false,false>")
            if n == 256 else None,
            "basis": "44 B per update (state read and written, three FP32 acceleration "
                     "fields read); one step per launch on the single-step tile kernel"}


def _thermal_leg(args, L, wl, dev, stream, drho_t, u_t, n):
    """The 256^3 Taylor-Green step with a temperature field advected by the
    flow (lwacm_set_thermal, omega_t = 1.4): the temperature step runs inside
    the single-step flow tile kernel (T read and written beside the state: 40
    B per node against 32 for the flow alone).  Timed beside the same steps
    without T, on the same kernel."""
    import torch
    cfg = wl.TGV3D_256
    times = []
    for thermal in (False, True):
        s9 = L.Solver(L.LWACM_D3Q19, n, n, n, cfg.omega, device=dev, variant=2)
        s9.set_state(drho_t, u_t)
        if thermal:
            s9.set_thermal(1.4, 0.5 + 0.5 * torch.rand((n, n, n), device=dev))
        s9.step(args.warmup)
        times.append(_events_time(s9.step, args.steps, stream))
        s9.close()
    torch.cuda.empty_cache()
    ms_flow, ms_both = (t / args.steps * 1e3 for t in times)
    nodes = n ** 3
    print(f"[bench] thermal {n}^3: {ms_both:.4f} ms/step with T, {ms_flow:.4f} without",
          file=sys.stderr, flush=True)
    fused = n % 32 == 0
    kname = "k_fwd_march_rolled<float,128,false,false,false,0,false,true>"
    return {"value": round(nodes * args.steps / times[1] / 1e6, 1),
            "unit": "MLUPS (flow and temperature)", "ms_per_step": round(ms_both, 5),
            "ms_flow_only": round(ms_flow, 5), "ms_added_by_temperature": round(ms_both - ms_flow, 5),
            "achieved_GBs": round(40.0 * nodes / (ms_both * 1e-3) / 1e9, 1),
            "kernel": kname if fused else "k_thermal_step<19,false> + k_fwd_march_rolled",
            "traffic": _measured_traffic(kname) if n == 256 else None,
            "basis": "40 B per node: FP32 flow state and T read and written in one pass"}


def _thermal_cavity_leg(args, L, wl, dev, stream):
    """The 192^3 lid-driven cavity with a temperature field: the walls at rest
    held at T = 0.2, the lid at T = 0.8 (omega_t = 1.4).  The temperature step
    runs inside the masked single-step flow kernel: per node 52 B (the state
    read and written, the link set, T read and written, the node's 8-byte entry
    of the fixed-temperature wall table).  Timed beside the same steps
    without T on the same kernel."""
    import torch
    c4 = wl.CAVITY_192
    m4 = torch.as_tensor(wl.cavity_mask(c4.nx), device=dev)
    shape = (c4.nz, c4.ny, c4.nx)
    times = []
    for thermal in (False, True):
        s = L.Solver(L.LWACM_D3Q19, c4.nx, c4.ny, c4.nz, c4.omega, mask=m4,
                     wall_u=[list(r) for r in wl.wall_table(c4.lid)], device=dev, variant=2)
        s.set_state(torch.zeros(shape, device=dev), torch.zeros((3,) + shape, device=dev))
        if thermal:
            s.set_thermal(1.4, torch.full(shape, 0.5, device=dev),
                          wall_T=[float("nan"), 0.2, 0.8])
        s.step(args.warmup)
        times.append(_events_time(s.step, args.steps, stream))
        s.close()
    torch.cuda.empty_cache()
    ms_flow, ms_both = (t / args.steps * 1e3 for t in times)
    fluid = (c4.nx - 2) * (c4.ny - 2) * (c4.nz - 2)
    print(f"[bench] cavity 192^3 with T: {ms_both:.4f} ms/step, {ms_flow:.4f} without",
          file=sys.stderr, flush=True)
    return {"value": round(fluid * args.steps / times[1] / 1e6, 1),
            "unit": "MLUPS (fluid nodes, flow and temperature)", "ms_per_step": round(ms_both, 5),
            "ms_flow_only": round(ms_flow, 5),
            "ms_added_by_temperature": round(ms_both - ms_flow, 5),
            "achieved_GBs": round(52.0 * c4.nx * c4.ny * c4.nz / (ms_both * 1e-3) / 1e9, 1),
            "kernel": "k_fwd_march_rolled<float,64,false,true,false,0,false,true>",
            "basis": "52 B per node: state in and out, link set, T in and out, wall-table entry; "
                     "one step per launch (the two-step kernel does not carry T)"}


def _c5_leg(L, wl, dev):
    """End-to-end gradient of the D2Q9 512^2 workload (seeded k <= 8 fields,
    omega 1.6, loss sum |u_T - u*|^2): 2000 forward steps storing a checkpoint
    every 100, then the reverse sweep (recompute each segment, 2000 reverse
    steps); host-synchronised wall time of each half."""
    import torch
    from paper_1111_2142_amd.autograd import lwacm_run
    c5 = wl.ADJOINT_512
    d5, u5 = wl.divergence_free_field(c5.nx, 8, c5.u0, seed=0)
    _, ut5 = wl.divergence_free_field(c5.nx, 8, c5.u0, seed=1)
    tgt = torch.as_tensor(ut5, dtype=torch.float64, device=dev)
    times = []
    for _ in range(2):  # the first run warms the kernels and the allocator
        d_t = torch.as_tensor(d5, dtype=torch.float32, device=dev).requires_grad_(True)
        u_t = torch.as_tensor(u5, dtype=torch.float32, device=dev).requires_grad_(True)
        om = torch.tensor(c5.omega, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, u_T = lwacm_run(d_t, u_t, om, c5.steps, L.LWACM_D2Q9, K=100)
        loss = ((u_T.double() - tgt) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fw, bw = times[-1]
    print(f"[bench] gradient 512^2 x 2000 steps (K = 100): forward {fw * 1e3:.1f} ms, "
          f"reverse sweep {bw * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"steps": c5.steps, "checkpoint_every": 100, "forward_ms": round(fw * 1e3, 2),
            "reverse_sweep_ms": round(bw * 1e3, 2), "total_ms": round((fw + bw) * 1e3, 2),
            "reverse_over_forward": round(bw / fw, 3), "loss": loss.item(),
            "dL_domega": float(om.grad),
            "basis": "host-synchronised wall time; the reverse sweep recomputes each "
                     "100-step segment from its checkpoint and runs 2000 reverse steps "
                     "(launch-bound at this size)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--variant", type=int, default=0,
                    help="0 auto, 1 generic, 2 march (one step per launch), 3 march2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forward-only", action="store_true",
                    help="time only the forward step of the 256^3 workload (for profiler runs)")
    ap.add_argument("--storage", choices=["fp32", "fp16"], default="fp32",
                    help="storage of the --forward-only run")
    ap.add_argument("--reverse-only", action="store_true",
                    help="time only the reverse (adjoint) step of the 256^3 workload (two per "
                         "launch; --variant 2: one per launch)")
    ap.add_argument("--split-only", action="store_true",
                    help="time only the 256^3 step with a separate omega_p (nu_p = 10 nu)")
    ap.add_argument("--qbb-only", action="store_true",
                    help="time only the 192^3 cavity with interpolated bounce-back (q = 0.3)")
    ap.add_argument("--field-only", action="store_true",
                    help="time only the 256^3 step with a node-by-node acceleration field")
    ap.add_argument("--thermal-cavity-only", action="store_true",
                    help="time the 192^3 cavity with a temperature field and exit")
    ap.add_argument("--thermal-only", action="store_true",
                    help="time only the 256^3 step with a temperature field")
    ap.add_argument("--cavity-only", action="store_true",
                    help="time only the 192^3 lid-driven cavity (walls, moving lid)")
    ap.add_argument("--stream-reference", action="store_true",
                    help="time the hand-written streaming kernels of bench_stream_ref.hip "
                         "(16-byte buffer copy, read and write of 1 GiB under four cache "
                         "policies): the HBM rate the HBM-bound steps are read against")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of 256 MiB (the reference kernel for "
                         "scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo-exchange design is described but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1111_2142_amd import lwacm as L

    L.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.stream_reference:
        print(json.dumps({"stream_reference": _stream_reference(dev)}), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        dt = _events_time(lambda k: [dst.copy_(src) for _ in range(k)], args.steps, stream)
        nbytes = 2 * src.numel() * 4
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": args.steps,
                          "ms_per_launch": dt / args.steps * 1e3,
                          "GBs": nbytes * args.steps / dt / 1e9}), flush=True)
        return
    if args.qbb_only:
        print(json.dumps({"cavity_192_interpolated": _qbb_leg(args, L, wl, dev, stream)}),
              flush=True)
        return
    if args.cavity_only:
        print(json.dumps({"cavity_192": _cavity_leg(args, L, wl, dev, stream)}), flush=True)
        return
    if args.thermal_cavity_only:
        print(json.dumps({"thermal_cavity_192": _thermal_cavity_leg(args, L, wl, dev, stream)}),
              flush=True)
        return
    n = args.n
    cfg = wl.TGV3D_256
    drho, u = wl.taylor_green_3d(n, cfg.u0)
    drho_t = torch.as_tensor(drho, dtype=torch.float32, device=dev)
    u_t = torch.as_tensor(u, dtype=torch.float32, device=dev)
    nodes = n ** 3
    del drho, u
    if args.field_only:
        print(json.dumps({"force_field": _field_leg(args, L, wl, dev, stream, drho_t, u_t, n)}),
              flush=True)
        return
    if args.thermal_only:
        print(json.dumps({"thermal": _thermal_leg(args, L, wl, dev, stream, drho_t, u_t, n)}),
              flush=True)
        return
    if args.split_only:
        print(json.dumps({"omega_p_split": _split_leg(args, L, wl, dev, stream, drho_t, u_t, n)}),
              flush=True)
        return

    def make(storage, rounding=L.LWACM_ROUND_STOCHASTIC):
        s = L.Solver(L.LWACM_D3Q19, n, n, n, cfg.omega, storage=storage, device=dev,
                     variant=args.variant, fp16_rounding=(rounding, 0))
        s.set_state(drho_t, u_t)
        return s

    if args.reverse_only:
        s = make(L.LWACM_FP32)
        s.step(2)
        st = s.save_state()
        s.step(1)
        st2 = s.save_state()  # the state of the step after st: two distinct inputs
        mu_a = torch.zeros((4, n, n, n), dtype=torch.float32, device=dev)
        mu_b = torch.zeros_like(mu_a)
        lam = torch.zeros_like(mu_a)
        lam[1:] = u_t
        dw = torch.zeros(1, dtype=torch.float64, device=dev)
        L.lwacm_adjoint_seed(s.ctx, st, lam, mu_a)

        two = args.variant in (0, 3)

        def rev(k):
            a_, b_ = mu_a, mu_b
            if two:
                for _ in range(k // 2):
                    if not L.lwacm_adjoint_step2(s.ctx, st2, st, a_, b_, dw, False):
                        raise RuntimeError("two-step reverse kernel declined the 256^3 problem")
                    a_, b_ = b_, a_
            else:
                for _ in range(k):
                    L.lwacm_adjoint_step(s.ctx, st, a_, b_, dw, False)
                    a_, b_ = b_, a_

        rev(args.warmup)
        dt = _events_time(rev, args.steps, stream)
        print(f"[bench] reverse step: {dt / args.steps * 1e3:.4f} ms/step", file=sys.stderr,
              flush=True)
        return

    if args.forward_only and args.storage == "fp16":
        s16 = make(L.LWACM_FP16_DEV)
        s16.step(args.warmup)
        dt = _events_time(s16.step, args.steps, stream)
        print(f"[bench] fp16 forward: {dt / args.steps * 1e3:.4f} ms/step", file=sys.stderr,
              flush=True)
        return

    # ---- FP32 forward (the headline)
    s32 = make(L.LWACM_FP32)
    s32.step(args.warmup)
    dt32_ev = _events_time(s32.step, args.steps, stream)
    ms32 = dt32_ev / args.steps * 1e3
    mlups32 = nodes * args.steps / dt32_ev / 1e6
    mass, energy = s32.diagnostics()
    print(f"[bench] fp32 forward: {ms32:.4f} ms/step, {mlups32:.0f} MLUPS, mass {mass:.6f}, "
          f"energy {energy:.6e}", file=sys.stderr, flush=True)

    fused = n == 256 and args.variant in (0, 3) and args.steps % 2 == 0
    kname = "k_fwd_march2<128,false>" if fused else "k_fwd_march_rolled<float,128,false,false,false,0,false,false>"
    per_launch = 2 if fused else 1
    vi = _measured(kname, "valu_insts_per_launch") if n == 256 else None
    traffic = _measured_traffic(kname) if n == 256 else None

    def roof(ms_step):
        """The dominant kernel's rooflines at ms_step milliseconds per step (the
        event time of back-to-back launches divided by the updates per launch)."""
        t_launch = ms_step * 1e-3 * per_launch
        tf = FLOPS_PER_UPDATE * nodes * per_launch / t_launch / 1e12
        eff = 32.0 * nodes / (ms_step * 1e-3) / 1e9
        return {"ms_per_step": round(ms_step, 5), "launch_us": round(t_launch * 1e6, 2),
                "achieved": round(tf, 3), "frac": round(tf / FP32_UNPACKED_TFLOPS, 4),
                "frac_of_packed_peak": round(tf / FP32_PEAK_TFLOPS, 4),
                "valu_issue_frac": None if vi is None else
                round(vi / (VALU_WAVE_INSTS_PER_S * t_launch), 4),
                "hbm_GBs_measured": None if traffic is None else round(traffic / t_launch / 1e9, 1),
                "hbm_frac_measured": None if traffic is None else
                round(traffic / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                "single_step_equivalent_GBs": round(eff, 1),
                "single_step_equivalent_frac": round(eff / HBM_PEAK_GBS, 4)}

    # the same kernel over a sustained run (the clock settles lower under
    # continuous VALU load than in a short burst)
    n_sus = 400
    dt_sus = _events_time(s32.step, n_sus, stream)
    burst, sustained = roof(ms32), roof(dt_sus / n_sus * 1e3)
    sustained["steps"] = n_sus
    print(f"[bench] fp32 forward sustained ({n_sus} steps): {sustained['ms_per_step']:.4f} "
          f"ms/step", file=sys.stderr, flush=True)
    result = {
        "metric": METRIC,
        "value": round(mlups32, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"d3q19_tgv_{n}^3", "lattice": "D3Q19", "grid": [n, n, n],
                   "omega": cfg.omega, "u0": cfg.u0, "storage": "fp32",
                   "diagnostics": "fused FP64 mass+energy every step"},
        "roofline": {"bound": "alu", "achieved": burst["achieved"],
                     "peak": FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s", "frac": burst["frac"],
                     "traffic": traffic, "kernel": kname if n == 256 else None,
                     "flops_per_update": FLOPS_PER_UPDATE, "updates_per_launch": per_launch,
                     "algorithmic_flops_per_launch": FLOPS_PER_UPDATE * nodes * per_launch,
                     "launch_us": burst["launch_us"],
                     "peak_basis": "FP32 FMA on every lane of 256 CUs x 4 SIMDs x 16 lanes at "
                                   "2.4 GHz (78.6 TFLOP/s); the published 157.3 counts packed "
                                   "FP32, which the kernels do not use",
                     "frac_of_packed_peak": burst["frac_of_packed_peak"],
                     "valu_issue_frac": burst["valu_issue_frac"],
                     "hbm_GBs_measured": burst["hbm_GBs_measured"],
                     "hbm_frac_measured": burst["hbm_frac_measured"],
                     "single_step_equivalent_GBs": burst["single_step_equivalent_GBs"],
                     "single_step_equivalent_frac": burst["single_step_equivalent_frac"],
                     "basis": "achieved = 157 FP32 operations per lattice update x updates "
                              "per launch / launch time (HIP events over the timed steps on "
                              "the library's stream); the kernel runs two steps per pass "
                              "(16 B of HBM per update: traffic) and is bound by VALU issue "
                              "(valu_issue_frac from the committed instruction counter); "
                              "single_step_equivalent: 32 B per update (one state read and "
                              "one write, the single-step minimum) against 8 TB/s",
                     "sustained": sustained},
    }
    if args.forward_only:
        print(json.dumps(result), flush=True)
        return

    # ---- the single-step tile kernel (32 B of HBM per update)
    s1 = L.Solver(L.LWACM_D3Q19, n, n, n, cfg.omega, device=dev, variant=L.LWACM_KERNEL_MARCH)
    s1.set_state(drho_t, u_t)
    s1.step(args.warmup)
    dt1 = _events_time(s1.step, args.steps, stream)
    s1.close()
    ms1 = dt1 / args.steps * 1e3
    print(f"[bench] fp32 single-step kernel: {ms1:.4f} ms/step", file=sys.stderr, flush=True)
    result["single_step"] = {
        "value": round(nodes * args.steps / dt1 / 1e6, 1), "unit": "MLUPS",
        "ms_per_step": round(ms1, 5),
        "achieved_GBs": round(32.0 * nodes / (ms1 * 1e-3) / 1e9, 1),
        "frac": round(32.0 * nodes / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernel": "k_fwd_march_rolled<float,128,false,false,false,0,false,false>" if n == 256 else None,
        "traffic": _measured_traffic("k_fwd_march_rolled<float,128,false,false,false,0,false,false>")
        if n == 256 else None}

    # ---- FP16-deviation storage
    s16 = make(L.LWACM_FP16_DEV)
    s16.step(args.warmup)
    dt16 = _events_time(s16.step, args.steps, stream)
    ms16 = dt16 / args.steps * 1e3
    mlups16 = nodes * args.steps / dt16 / 1e6
    print(f"[bench] fp16 forward: {ms16:.4f} ms/step, {mlups16:.0f} MLUPS", file=sys.stderr,
          flush=True)
    s16.close()
    s16n = make(L.LWACM_FP16_DEV, L.LWACM_ROUND_NEAREST)
    s16n.step(args.warmup)
    dt16n = _events_time(s16n.step, args.steps, stream)
    s16n.close()
    result["fp16_store"] = {"value": round(mlups16, 1), "unit": "MLUPS",
                            "ms_per_step": round(ms16, 5), "rounding": "stochastic (pcg2d words, hardware conversion)",
                            "achieved_GBs": round(16.0 * nodes / dt16 * args.steps / 1e9, 1),
                            "ms_per_step_nearest_rounding": round(dt16n / args.steps * 1e3, 5),
                            "kernel": "k_fwd_march_rolled<__half,128,true,false,false,0,false,false>"
                            if n == 256 else None,
                            "traffic": _measured_traffic("k_fwd_march_rolled<__half,128,true,false,false,0,false,false>")
                            if n == 256 else None}

    # ---- reverse step at the same size (reads state_t and mu_t, writes mu_{t-1});
    # two per launch: the states of two consecutive steps (distinct buffers)
    st = s32.save_state()
    s32.step(1)
    st2 = s32.save_state()
    mu_a = torch.zeros((4, n, n, n), dtype=torch.float32, device=dev)
    mu_b = torch.zeros_like(mu_a)
    dw = torch.zeros(1, dtype=torch.float64, device=dev)
    lam = torch.zeros_like(mu_a)
    lam[1:] = u_t
    L.lwacm_adjoint_seed(s32.ctx, st, lam, mu_a)
    nadj = 2 * max(5, args.steps // 8)  # even: the sweep runs two reverse steps per launch

    def adj(k, two=True):
        a, b = mu_a, mu_b
        if two:
            for _ in range(k // 2):
                if not L.lwacm_adjoint_step2(s32.ctx, st2, st, a, b, dw, False):
                    raise RuntimeError("two-step reverse kernel declined the problem")
                a, b = b, a
        else:
            for _ in range(k):
                L.lwacm_adjoint_step(s32.ctx, st, a, b, dw, False)
                a, b = b, a

    adj(4)
    dta = _events_time(adj, nadj, stream)
    msa = dta / nadj * 1e3
    adj(4, False)
    dta1 = _events_time(lambda k: adj(k, False), nadj, stream)
    msa1 = dta1 / nadj * 1e3
    print(f"[bench] reverse step: {msa:.4f} ms/step (two per launch), {msa1:.4f} ms one per "
          f"launch", file=sys.stderr, flush=True)
    result["adjoint"] = {"ms_per_step": round(msa, 5),
                         "adjoint_forward_ratio": round(msa / ms32, 3),
                         "with_recompute_ratio": round((msa + ms32) / ms32, 3),
                         "achieved_GBs": round(32.0 * nodes / (msa * 1e-3) / 1e9, 1),
                         "basis": "reverse steps two per launch (lwacm_adjoint_step2): state_t, "
                                  "state_t-1, mu in, mu out = 32 B per node and step",
                         "kernel": "k_adj_march2<float,false,128>" if n == 256 else None,
                         "traffic": _measured_traffic("k_adj_march2<float,false,128>")
                         if n == 256 else None,
                         "one_step_kernel": {
                             "ms_per_step": round(msa1, 5),
                             "adjoint_forward_ratio": round(msa1 / ms32, 3),
                             "ratio_to_single_step_forward": round(msa1 / ms1, 3),
                             "achieved_GBs": round(48.0 * nodes / (msa1 * 1e-3) / 1e9, 1),
                             "kernel": "k_adj_march<float,false>" if n == 256 else None,
                             "traffic": _measured_traffic("k_adj_march<float,false>")
                             if n == 256 else None}}
    s32.close()
    del mu_a, mu_b, lam, st, st2
    torch.cuda.empty_cache()
    dw.zero_()

    # ---- lid-driven cavity 192^3 (mask active, moving lid)
    result["cavity_192"] = _cavity_leg(args, L, wl, dev, stream)

    # ---- separate omega_p for the density: the same 256^3 step, one step per launch
    result["omega_p_split"] = _split_leg(args, L, wl, dev, stream, drho_t, u_t, n)

    # ---- node-by-node body acceleration: the same 256^3 step
    result["force_field"] = _field_leg(args, L, wl, dev, stream, drho_t, u_t, n)

    # ---- temperature advected by the flow: the same 256^3 step plus the temperature kernel
    result["thermal"] = _thermal_leg(args, L, wl, dev, stream, drho_t, u_t, n)
    # ---- the same with walls: the 192^3 cavity with hot lid and cold walls
    result["thermal_cavity_192"] = _thermal_cavity_leg(args, L, wl, dev, stream)

    # ---- interpolated bounce-back: the 192^3 cavity with walls at q = 0.3
    result["cavity_192_interpolated"] = _qbb_leg(args, L, wl, dev, stream)

    # ---- differentiable D2Q9 512^2: reverse / forward at the gradient workload (launch-bound)
    c5 = wl.ADJOINT_512
    s5 = L.Solver(L.LWACM_D2Q9, c5.nx, c5.ny, 1, c5.omega, device=dev)
    d5, u5 = wl.divergence_free_field(c5.nx, 8, c5.u0, seed=0)
    s5.set_state(torch.as_tensor(d5, dtype=torch.float32, device=dev),
                 torch.as_tensor(u5, dtype=torch.float32, device=dev))
    s5.step(args.warmup)
    dt5f = _events_time(s5.step, args.steps, stream)
    st5 = s5.save_state()
    m5a = torch.zeros((3, 1, c5.ny, c5.nx), dtype=torch.float32, device=dev)
    m5b = torch.zeros_like(m5a)
    lam5 = torch.zeros_like(m5a)
    lam5[1:] = torch.as_tensor(u5, dtype=torch.float32, device=dev)
    L.lwacm_adjoint_seed(s5.ctx, st5, lam5, m5a)

    def adj5(k):
        a, b = m5a, m5b
        for _ in range(k):
            L.lwacm_adjoint_step(s5.ctx, st5, a, b, dw, False)
            a, b = b, a

    adj5(3)
    dt5a = _events_time(adj5, args.steps, stream)
    # the reverse steps as a checkpointed sweep runs them: the segment's states
    # recomputed into slots, then lwacm_adjoint_sweep (up to 8 steps per launch)
    sb5 = s5.state_bytes
    seg5 = torch.empty(args.steps * sb5, dtype=torch.uint8, device=dev)
    seg5[:sb5].copy_(st5)
    if args.steps > 1:
        L.lwacm_forward_states(s5.ctx, st5, 0, args.steps - 1, seg5[sb5:])

    def sweep5(k):  # a segment after the first (t0 > 0: mu stays node-interleaved)
        L.lwacm_adjoint_sweep(s5.ctx, seg5, 1, k, m5a, m5b, dw)

    sweep5(args.steps)  # allocates the sweep's partial buffers once
    dt5s = _events_time(sweep5, args.steps, stream)
    s5.close()
    result["adjoint_d2q9_512"] = {
        "forward_ms": round(dt5f / args.steps * 1e3, 5),
        "reverse_ms": round(dt5s / args.steps * 1e3, 5),
        "adjoint_forward_ratio": round(dt5s / dt5f, 3),
        "reverse_ms_one_per_launch": round(dt5a / args.steps * 1e3, 5),
        "basis": "forward: lwacm_step (up to 8 steps per launch); reverse: "
                 "lwacm_adjoint_sweep over the same number of stored states (up to 8 "
                 "per launch), as the checkpointed gradient runs it; one_per_launch: "
                 "lwacm_adjoint_step calls"}
    print(f"[bench] d2q9 512^2: forward {dt5f / args.steps * 1e3:.4f} ms, reverse "
          f"{dt5s / args.steps * 1e3:.4f} ms (sweep), {dt5a / args.steps * 1e3:.4f} ms one per "
          f"launch", file=sys.stderr, flush=True)

    # ---- the differentiable workload at its configured length: 2000 forward
    # steps with a checkpoint every 100, then the checkpointed reverse sweep
    result["gradient_d2q9_512"] = _c5_leg(L, wl, dev)

    # ---- FP64 CPU oracle on a bounded sample of the same workload
    if not args.no_cpu_baseline:
        import oracle
        p = oracle.Problem(q=19, nx=n, ny=n, nz=n, omega=cfg.omega)
        d0, u0 = wl.taylor_green_3d(n, cfg.u0)
        r0 = 1.0 + d0
        del d0
        oracle.run(p, r0, u0, 1)   # warm-up (page-in)
        nsteps_cpu = 24
        threads = oracle.num_threads()
        t0 = time.perf_counter()
        oracle.run(p, r0, u0, nsteps_cpu)
        dtc = time.perf_counter() - t0
        # the same update on one thread, one step
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        oracle.run(p, r0, u0, 1)
        dt1 = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        cpu_model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        result["cpu_baseline"] = {
            "value": round(nodes * nsteps_cpu / dtc / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model,
            "host_cpus_visible": os.cpu_count(),
            "sample": f"{nsteps_cpu} steps of the full {n}^3 D3Q19 Taylor-Green grid "
                      "(FP64, OpenMP over z-y rows); single_thread: 1 step on 1 thread",
            "single_thread": round(nodes / dt1 / 1e6, 3)}
        print(f"[bench] cpu oracle: {result['cpu_baseline']['value']} MLUPS on "
              f"{oracle.num_threads()} threads", file=sys.stderr, flush=True)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
