"""Benchmark: frames/s of tiDAS vs DAS at 256 x 1024 px with 128 channels.

Workload (clinical-size plain case): 128-element linear array, 0.3 mm pitch,
7.5 MHz 2-cycle pulse, 50 MHz sampling, 4096 float32 samples per channel,
one 0-degree plane wave; per frame a speckle phantom of 100k scatterers in
38 x 60 mm with 5 anechoic cysts (per-frame seed); image 256 lateral x 1024
depth; tiDAS with 129-tap exact-mode row kernels.

One step = one batch of B frames through the hot path: the tiDAS line model
(tidas_apply) over the B reflectivity maps, and exact DAS (das_beamform) over
the B RF records of the same phantoms.  Inputs are resident in HBM before the
timed regions.  ``value`` is tiDAS frames/s; DAS frames/s and the speedup are
reported beside it, each with its rel-L2 against the FP64 oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]

Other workloads (one JSON line each, not the headline):
    --workload batch    64 ragged frames (256..512 x 512..2048 px), 11 compounded
                        plane waves, 64-element array: one persistent launch per
                        batch (autotuned variant) vs 64 per-frame launches, for DAS
                        and the line model
    --workload deconv   200 Tikhonov gradient iterations on a 256 x 1024 map
                        (500 spikes, 40 dB noise, lambda 1e-3, 65 taps)
    --workload approx   the paper-style 1-D approximation error (on-axis line,
                        plane wave): single scatterers at every row and 5 / 5 rising /
                        100 scatterer lines, exact kernels and one reference curve
                        at 25 and 35 mm, local and global squared errors
    --workload beamform the paper's time-invariant beamformer from RF (tidas_beamform:
                        receive law frozen per neighbourhood of rows, theta from paper
                        mode) vs exact DAS on the benchmark's 64 speckle frames: frames/s,
                        rel-L2 vs the oracle, 2-D error against DAS
    --workload separable  the separable 2-D extension: the line model's depth pass
                        followed by a lateral per-row pass (tidas_apply_lateral) on the
                        benchmark's 64 frames: time, HBM roofline of the lateral pass,
                        2-D error against DAS with and without the lateral pass
    --workload kgrad    gradient of the line model in its kernels (tidas_kernel_grad)
                        over B frames of 1024 x 256 with 129 taps
    --workload study    the paper's single-point study (tidas_point_study): 600 points
                        from 2 to 42 mm, focused transmit with a Kossoff aperture at
                        15 / 25 / 35 mm, 3-9 MHz; Theta matrix and local / global error
                        maps of all 360k (delay curve, scatterer) pairs per setting,
                        DAS / tiDAS peak ratios and FWHM differences
    --workload surrogate  train the BF16-MFMA kernel surrogate on 200k exact
                        kernels (depth, F# 1-3, angle +-15 deg, fc 3-10 MHz), then
                        surrogate-kernel vs exact-kernel line model on 512 x 2048
                        speckle (129 taps): rel-L2, bank generation and frames/s
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks, and the derived fp32 FMA ceiling of this build's VALU code
HBM_PEAK_GBS = 8000.0
FP32_VALU_NOPACK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6: 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz
# DAS work per active (pixel, element, angle) term, counted from the definition:
# receive distance 4 (sub, mul, add, sqrt), index 2, interpolation 3, apodization 3
# (scale, cos, add), weighted accumulate 2
DAS_FLOPS_PER_TERM = 14


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["main", "batch", "deconv", "beamform", "separable", "kgrad", "surrogate",
                                           "approx", "study"],
                    default="main")
    ap.add_argument("--train-steps", type=int, default=20000, help="surrogate workload: Adam steps")
    ap.add_argument("--train-rows", type=int, default=200_000, help="surrogate workload: training kernels")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=64, help="frames per step")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle parity check")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--cpu-single-core", action="store_true",
                    help="time the CPU oracle on one core only (no worker processes)")
    ap.add_argument("--only", choices=["tidas", "das"], default=None, help="time one op only (profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run one plain device copy of known byte count (main: the input batch; batch: 64 MiB) so "
                         "hardware byte counters can be calibrated against it")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tidas_b4_kernel_256x1024_k129_b64_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tidas_b4_batch_kernel_ragged64_k65_traffic.json")
LATERAL_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lateral_pass_kernel_1024x256_k33_b64_traffic.json")
BF16_MFMA_TFLOPS = 2500.0                                    # dense bf16 matrix peak
FP32_MFMA_TFLOPS = 157.3                                     # dense fp32 matrix peak


def measured_traffic(batch, path=TRAFFIC_FILE):
    """HBM bytes per launch of the line-model kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by a plain copy of known
    size), or None when the kernel source changed since they were taken or the
    batch differs from the profiled one."""
    import hashlib
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if sha != rec.get("source_sha256") or batch != 64:
        return None
    return rec["traffic_bytes_per_launch"]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    {"main": run_main, "batch": run_batch, "deconv": run_deconv, "beamform": run_beamform,
     "separable": run_separable, "kgrad": run_kgrad,
     "surrogate": run_surrogate,
     "approx": run_approx, "study": run_study}[args.workload](args)


def _oracle_apply_frames(task):
    """One worker task of the pooled CPU baseline: the oracle line model on a
    batch of frames (runs in a process forked before the GPU is touched)."""
    from oracle import tidas as o_t
    kb, R = task
    o_t.apply(kb, R)
    return R.shape[0]


def _cpu_pool():
    """Worker processes for the CPU baseline, forked before anything
    initialises the GPU (they never touch it, and they have exited before the
    GPU work starts): one per host core the job may use, at most 16.  None
    when the host has a single core."""
    import multiprocessing
    n = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1))
    if n < 2:
        return None
    return multiprocessing.get_context("fork").Pool(n)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _main_oracle_inputs(s, phantoms, K):
    """Host-side inputs of the oracle for the main workload, from the seeded
    generators and the oracle itself (never from device results): the FP64
    exact bank, the reflectivity maps of frames 0-3 and the RF of frame 0."""
    import numpy as np

    from oracle import kernels as o_k, simulate as o_sim
    from workloads import generators
    Z, X = s.nz, s.nx
    xs = s.x0 + np.arange(X) * s.dx
    zs = s.z0 + np.arange(Z) * s.dz
    okw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
               n_samples=s.n_samples, angles=list(s.angles))
    dkw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, angles=list(s.angles), fnumber=s.fnumber)
    kb_o = o_k.exact_kernels(zs, s.dz, K, fnumber=s.fnumber, **okw)
    R_host = []
    for b in range(4):
        xb, zb, ab = phantoms[b]
        ib, jb, _, _ = generators.snap_to_grid(xb, zb, s.x0, s.dx, X, s.z0, s.dz, Z)
        R_host.append(generators.reflectivity_map(ib, jb, ab, Z, X).astype(np.float32))
    x, z, a = phantoms[0]
    rf_o = o_sim.to_fp32(o_sim.simulate_rf(x, z, a, **okw))
    return dict(kb_o=kb_o, R_host=np.stack(R_host), rf_o=rf_o, xs=xs, zs=zs, dkw=dkw)


def _main_cpu_baselines(host, single_core):
    """The oracle timed on the host's cores, before the GPU is touched: the
    line model over a pool of worker processes (one batch of 4 frames per task,
    about 12 s), the line model on one core (about 12 s) and DAS on one core
    (about 8 s).  The workers exit before this returns."""
    import numpy as np

    from oracle import das as o_das, tidas as o_t
    kb_o, Rc = host["kb_o"], host["R_host"].astype(np.float64)
    res = {}
    pool = None if single_core else _cpu_pool()
    if pool is not None:
        n_w = pool._processes
        tasks = [(kb_o, Rc)] * n_w
        n_fr, t_c = 0, time.perf_counter()
        while time.perf_counter() - t_c < 12.0:
            n_fr += sum(pool.map(_oracle_apply_frames, tasks))
        res["pool"] = {"value": n_fr / (time.perf_counter() - t_c), "unit": "frames/s", "cores": n_w,
                       "kind": "oracle",
                       "sample": f"FP64 oracle line model on {n_fr} frames of the workload over {n_w} worker "
                                 f"processes (batches of 4 frames), about 12 s"}
        pool.close()
        pool.join()
    n_fr, t_c = 0, time.perf_counter()
    while time.perf_counter() - t_c < 12.0:
        o_t.apply(kb_o, Rc)
        n_fr += Rc.shape[0]
    res["single"] = {"value": n_fr / (time.perf_counter() - t_c), "unit": "frames/s", "cores": 1,
                     "kind": "oracle", "sample": f"FP64 oracle line model on {n_fr} frames of the workload "
                                                 f"(batches of 4), about 12 s"}
    n_d, t_c = 0, time.perf_counter()
    while time.perf_counter() - t_c < 8.0:
        o_das.das(host["rf_o"], host["xs"], host["zs"], **host["dkw"])
        n_d += 1
    res["das"] = {"value": n_d / (time.perf_counter() - t_c), "unit": "frames/s", "cores": 1,
                  "kind": "oracle", "sample": f"FP64 oracle DAS on {n_d} frames, about 8 s"}
    return res


def run_main(args):
    import numpy as np

    from workloads import config, generators
    from workloads.configs import CYSTS, N_SCATTERERS

    s = config(2)
    B, K = args.batch, s.K
    Z, X = s.nz, s.nx
    phantoms = []
    for b in range(B):
        x, z, a, _ = generators.speckle_with_cysts(N_SCATTERERS[2], s.field_w, s.field_d, CYSTS["n"], CYSTS["r_lo"],
                                                   CYSTS["r_hi"], seed=b)
        phantoms.append((x, z, a))
    # the oracle's inputs and the CPU baselines come first: the baseline's
    # worker processes are forked, timed and gone before torch touches the GPU
    host = cpu = None
    if not (args.no_parity and args.no_cpu_baseline):
        t_p = time.perf_counter()
        host = _main_oracle_inputs(s, phantoms, K)
        log(f"oracle inputs ready in {time.perf_counter() - t_p:.1f}s")
    if not args.no_cpu_baseline:
        cpu = _main_cpu_baselines(host, args.cpu_single_core)
        log("cpu baselines: " + ", ".join(f"{k} {v['value']:.2f} {v['unit']} on {v['cores']} cores"
                                          for k, v in cpu.items()))

    import torch

    import paper_2507_15464_amd as td

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # ---- inputs (untimed): per-frame phantoms, RF synthesised on the GPU, snapped reflectivity maps
    t_in = time.perf_counter()
    rf = torch.empty((B, 1, s.n_elem, s.n_samples), device=dev, dtype=torch.float32)
    R = torch.empty((B, Z, X), device=dev, dtype=torch.float32)
    for b in range(B):
        x, z, a = phantoms[b]
        scat = torch.tensor(np.stack([x, z, a], 1), dtype=torch.float64, device=dev)
        td.simulate_rf(s, scat, out=rf[b])
        i, j, _, _ = generators.snap_to_grid(x, z, s.x0, s.dx, X, s.z0, s.dz, Z)
        R[b] = torch.from_numpy(generators.reflectivity_map(i, j, a, Z, X).astype(np.float32))
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t_in:.1f}s")

    t_b = time.perf_counter()
    kb = td.build_kernels(s, mode="exact")
    prep = td.prepare(kb)  # per geometry, like the bank itself
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t_b
    Y = torch.empty_like(R)
    img = torch.empty((B, Z, X), device=dev, dtype=torch.float32)

    def run_tidas():
        td.apply(prep, R, out=Y)

    def run_tidas_unprepared():
        td.apply(kb, R, out=Y)

    def run_das():
        td.das_beamform(rf, s, out=img)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / args.steps, wall

    res = {}
    if args.only in (None, "tidas"):
        res["tidas"] = timed(run_tidas)
        log(f"tidas: {res['tidas'][0]:.4f} ms/step ({B} frames)")
    if args.only is None:
        res["tidas_unprepared"] = timed(run_tidas_unprepared)
        log(f"tidas (bank converted in the call): {res['tidas_unprepared'][0]:.4f} ms/step")
        # the adjoint (transpose) over the same frames, prepared bank
        res["adjoint"] = timed(lambda: td.adjoint(prep, R, out=Y))
        log(f"adjoint: {res['adjoint'][0]:.4f} ms/step")
    if args.only in (None, "das"):
        res["das"] = timed(run_das)
        log(f"das: {res['das'][0]:.4f} ms/step ({B} frames)")
    if args.only is None:
        # a plain device copy of the same bytes (read R, write Y): the HBM rate
        # this box reaches on a pure stream, beside the 8 TB/s peak
        res["copy"] = timed(lambda: Y.copy_(R))
        log(f"copy of the frames: {res['copy'][0]:.4f} ms/step")
    if args.copy_probe:
        Y.copy_(R)  # reads and writes exactly B*Z*X*4 bytes each
        torch.cuda.synchronize()
        log(f"copy probe: {R.numel() * 4} bytes read, {R.numel() * 4} bytes written")
    if args.only is not None:
        return

    tid_ms, das_ms = res["tidas"][0], res["das"][0]
    flops = 2.0 * K * Z * X * B                       # one FMA per tap per output pixel
    hbm_bytes = (8.0 * Z * X) * B + 4.0 * Z * K       # read R + write Y per frame, kernel bank once
    achieved_tflops = flops / (tid_ms * 1e-3) / 1e12
    achieved_gbs = hbm_bytes / (tid_ms * 1e-3) / 1e9
    # The line-model kernel the library picks for this launch (tidas_line_kernel):
    # the four-block tile (128 x 256) when its band window fits (K <= 161) and the
    # batch's tiles cover every compute unit, else the two-block tile (64 x 256).
    # Matrix work issued: per tile row and column, a window of 16 NSB (four-block:
    # NSB in 4..12 steps per 32-row block) or 16 NS rows (two-block: NS a multiple
    # of 4), six bf16 products per float32 product.
    need = (32 + K - 1 + 15) // 16
    nsb = next((n for n in (4, 6, 8, 10, 12) if n >= need), 0)
    cols = -(-X // 256) * 256
    if td.line_kernel(K, B, Z, X) == td._lib.LINE_FOUR_BLOCK:
        kernel = f"tidas_b4_kernel<false,{nsb},false,true>"
        mfma_flops = 2.0 * 6 * (16 * nsb) * (-(-Z // 128) * 128) * cols * B
    else:
        ns = ((64 + K - 1 + 15) // 16 + 3) // 4 * 4
        kernel = "tidas_bx6_kernel<false,true>"
        mfma_flops = 2.0 * 6 * (16 * ns) * (-(-Z // 64) * 64) * cols * B

    out = {
        "metric": "frames/s tiDAS vs DAS (256x1024 px, 128 ch) at stated rel-L2 vs FP64 oracle",
        "value": B / (tid_ms * 1e-3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tid_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 100k-scatterer speckle phantoms with cysts, RF synthesised on the GPU)",
        "config": {"workload": "tiDAS vs DAS, 128-ch plane wave, 256x1024 px image, 129-tap exact row kernels",
                   "frames_per_step": B, "channels": s.n_elem, "samples": s.n_samples, "image": [Z, X], "taps": K},
        "tidas": {"frames_per_s": B / (tid_ms * 1e-3), "mpixel_per_s": B * Z * X / (tid_ms * 1e-3) / 1e6,
                  "ms_per_step": tid_ms, "hbm_gbs_algorithmic": achieved_gbs,
                  "ms_per_step_bank_converted_in_call": res["tidas_unprepared"][0]},
        "das": {"frames_per_s": B / (das_ms * 1e-3), "mpixel_per_s": B * Z * X / (das_ms * 1e-3) / 1e6,
                "ms_per_step": das_ms},
        "tidas_speedup_vs_das": das_ms / tid_ms,
        "kernel_build_s": build_s,
        "adjoint": ({"ms_per_step": res["adjoint"][0], "frames_per_s": B / (res["adjoint"][0] * 1e-3),
                     "achieved_gbs": hbm_bytes / (res["adjoint"][0] * 1e-3) / 1e9} if "adjoint" in res else None),
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(B),
                     "kernel": kernel, "bytes_per_launch": hbm_bytes,
                     "copy_gbs_same_bytes": hbm_bytes / (res["copy"][0] * 1e-3) / 1e9 if "copy" in res else None,
                     "useful_fp32_tflops": achieved_tflops,
                     "mfma_bf16_tflops_issued": mfma_flops / (tid_ms * 1e-3) / 1e12,
                     "mfma_frac": mfma_flops / (tid_ms * 1e-3) / 1e12 / BF16_MFMA_TFLOPS},
    }

    # DAS terms per frame: (pixel, element) pairs inside the Hann aperture, times angles
    xs_h = s.x0 + np.arange(X) * s.dx
    zs_h = s.z0 + np.arange(Z) * s.dz
    xn_h = (np.arange(s.n_elem) - (s.n_elem - 1) / 2.0) * s.pitch
    half_ap = zs_h[:, None] / (2.0 * s.fnumber)
    terms = sum(int(np.count_nonzero(np.abs(xs_h[None, :] - x_n) <= half_ap)) for x_n in xn_h) * len(s.angles)
    das_tflops = DAS_FLOPS_PER_TERM * terms * B / (das_ms * 1e-3) / 1e12
    out["das"]["terms_per_frame"] = terms
    out["das_roofline"] = {"bound": "alu", "achieved": das_tflops, "peak": FP32_VALU_NOPACK_TFLOPS,
                           "unit": "TFLOP/s", "frac": das_tflops / FP32_VALU_NOPACK_TFLOPS,
                           "kernel": "das_interleave_kernel<4,2> + das_kernel<4,1,true>",
                           "flops_per_term": DAS_FLOPS_PER_TERM,
                           "note": "the call: interleaved copy and gathers; the gathers' address path bounds it"}

    # ---- tiDAS-vs-DAS approximation error on frame 0 (snapped phantom, both on the GPU)
    x, z, a = phantoms[0]
    i, j, zs_, xs_ = generators.snap_to_grid(x, z, s.x0, s.dx, X, s.z0, s.dz, Z)
    scat = torch.tensor(np.stack([xs_, zs_, a], 1), dtype=torch.float64, device=dev)
    rf_snap = td.simulate_rf(s, scat)
    d_snap = td.das_beamform(rf_snap, s)
    y_snap = td.apply(kb, R[0])
    out["approx_rel_l2_2d"] = float(torch.linalg.norm(y_snap - d_snap) / torch.linalg.norm(d_snap))
    # kernel-bank builds (once per geometry): exact mode, and paper mode with one
    # receive law per 64 rows
    t_b = time.perf_counter()
    td.build_kernels(s, mode="exact")
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t_b
    refs64 = [min((i // 64) * 64 + 32, Z - 1) for i in range(Z)]
    t_b = time.perf_counter()
    td.build_kernels(s, mode="paper", ref_row=refs64, with_theta=True)
    torch.cuda.synchronize()
    out["kernel_build_times_s"] = {"exact": t_exact, "paper_one_law_per_64_rows": time.perf_counter() - t_b}
    # the paper-style 1-D error on the centre line (single scatterers at every row, exact kernels)
    e1d = line_errors(s, K, dev)["exact"]
    out["approx_1d"] = {"single_local_sq_median": e1d["single_local_sq_median"],
                        "single_local_below_5pct": e1d["single_local_below_5pct"],
                        "single_global_sq_median": e1d["single_global_sq_median"],
                        "lines_global_sq": {p: e1d[p]["global_sq"] for p in ("5_uniform", "5_rising", "100_uniform")},
                        "paper_threshold": 0.05}

    if host is not None:
        from oracle import das as o_das, tidas as o_t
        kb_o, R_host, rf_o = host["kb_o"], host["R_host"], host["rf_o"]
        xs, zs, dkw = host["xs"], host["zs"], host["dkw"]

    if not args.no_parity:
        t_p = time.perf_counter()
        kb32 = kb_o.astype(np.float32)
        # the timed launch (all B frames, prepared bank) on the oracle's bank;
        # frames 0-3 of R are the maps of R_host (same seeded phantoms)
        y_all = td.apply(td.prepare(torch.from_numpy(kb32).to(dev)), R)
        assert torch.equal(R[:4].cpu(), torch.from_numpy(R_host))
        y_gpu = y_all[:4].cpu().numpy()
        y_ref = o_t.apply(kb32, R_host)
        out["tidas"]["rel_l2_vs_oracle"] = float(np.linalg.norm(y_gpu - y_ref) / np.linalg.norm(y_ref))
        out["tidas"]["parity_sample"] = f"frames 0-3 of the timed {B}-frame launch"
        out["kernel_bank_rel_l2_vs_oracle"] = float(np.linalg.norm(kb.cpu().numpy() - kb_o) / np.linalg.norm(kb_o))
        d_gpu = td.das_beamform(torch.from_numpy(rf_o).to(dev), s).cpu().numpy()
        d_ref = o_das.das(rf_o, xs, zs, **dkw)
        out["das"]["rel_l2_vs_oracle"] = float(np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref))
        log(f"parity done in {time.perf_counter() - t_p:.1f}s")

    if cpu is not None:
        # the all-core figure is the baseline; the one-core figures beside it
        out["cpu_baseline"] = cpu.get("pool", cpu["single"])
        out["cpu_baseline_single_core"] = cpu["single"]
        out["cpu_baseline_das"] = cpu["das"]
        out["cpu_model"] = _cpu_model()
    print(json.dumps(out), flush=True)


def _events_ms(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_batch(args):
    """64 ragged frames, 11 compounded angles: persistent batch launch vs per-frame launches."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads import config, generators
    from workloads.configs import RAGGED

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = config(3)
    sizes = generators.ragged_sizes(RAGGED["n_frames"], RAGGED["x_lo"], RAGGED["x_hi"], RAGGED["z_lo"],
                                    RAGGED["z_hi"], seed=0)
    t_in = time.perf_counter()
    grids, rfs, kbs, maps, outs_d, outs_t = [], [], [], [], [], []
    for f, (nz, nx) in enumerate(sizes):
        s = base.with_grid(nz, nx)
        x, z, a = generators.point_scatterers(20, s.field_w, s.field_d, seed=f)
        scat = torch.tensor(np.stack([x, z, a], 1), dtype=torch.float64, device=dev)
        grids.append(s)
        rfs.append(td.simulate_rf(s, scat))
        kbs.append(td.build_kernels(s, K=s.K, mode="exact"))
        i, j, _, _ = generators.snap_to_grid(x, z, s.x0, s.dx, nx, s.z0, s.dz, nz)
        maps.append(torch.from_numpy(generators.reflectivity_map(i, j, a, nz, nx).astype(np.float32)).to(dev))
        outs_d.append(torch.empty((nz, nx), device=dev))
        outs_t.append(torch.empty((nz, nx), device=dev))
    torch.cuda.synchronize()
    log(f"batch inputs ready in {time.perf_counter() - t_in:.1f}s")
    key = f"{len(sizes)}f_{sum(a * b for a, b in sizes)}px_A{len(base.angles)}_C{base.n_elem}_K{base.K}"
    v_das, das_times = td.autotune.tune("das_batch", lambda v: td.das_beamform_batch(base, grids, rfs, outs_d, v),
                                        key=key, force=True)
    v_app, app_times = td.autotune.tune("apply_batch", lambda v: td.apply_batch(kbs, maps, outs_t, v),
                                        key=key, force=True)
    n = len(sizes)
    das_batch = _events_ms(lambda: td.das_beamform_batch(base, grids, rfs, outs_d, v_das), args.steps, args.warmup)
    das_loop = _events_ms(lambda: [td.das_beamform(rfs[f], grids[f], out=outs_d[f]) for f in range(n)],
                          max(1, args.steps // 4), 1)
    app_batch = _events_ms(lambda: td.apply_batch(kbs, maps, outs_t, v_app), args.steps, args.warmup)
    # the batch prepared once (frame table and band images: per geometry, like
    # a bank), then one launch per step
    pb = td.PreparedBatch(kbs, maps, outs_t)
    app_prep = _events_ms(pb.apply, args.steps, args.warmup)
    app_loop = _events_ms(lambda: [td.apply(kbs[f], maps[f], out=outs_t[f]) for f in range(n)],
                          max(1, args.steps // 4), 1)
    if args.copy_probe:
        # a plain device copy of known size, for scaling the traffic counters
        src = torch.zeros(16 * 1024 * 1024, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {src.numel() * 4} bytes read, {src.numel() * 4} bytes written")
    px = sum(a * b for a, b in sizes)
    batch_bytes = float(sum(8 * a * b + 4 * a * base.K for a, b in sizes))
    out = {
        "metric": "frames/s, ragged 64-frame batch with 11-angle compounding (persistent launch vs per-frame)",
        "value": n / (app_prep * 1e-3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": app_prep, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (20-scatterer phantoms, per-frame seeds)",
        "config": {"workload": "64 ragged frames 256-512 x 512-2048 px, 11 angles -10..10 deg, 64 elements, K=65",
                   "pixels": px},
        "tidas": {"batch_ms": app_batch, "prepared_batch_ms": app_prep, "per_frame_launches_ms": app_loop,
                  "variant": v_app,
                  "variant_ms": app_times, "frames_per_s": n / (app_batch * 1e-3),
                  "launch_gain": app_loop / app_batch},
        "das": {"batch_ms": das_batch, "per_frame_launches_ms": das_loop, "variant": v_das,
                "variant_ms": das_times, "frames_per_s": n / (das_batch * 1e-3),
                "launch_gain": das_loop / das_batch},
        "tidas_speedup_vs_das": das_batch / app_prep,
        # the prepared batch's one launch: read every map, write every image,
        # read every bank once (8 Z X + 4 Z K bytes per frame)
        "roofline": {"bound": "hbm", "achieved": batch_bytes / (app_prep * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": batch_bytes / (app_prep * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(n, BATCH_TRAFFIC_FILE),
                     "kernel": "tidas_b4_kernel<false,6,true,true> (prepared batch)", "bytes_per_launch": batch_bytes},
    }
    print(json.dumps(out), flush=True)


def run_deconv(args):
    """200 Tikhonov gradient iterations through the line model on 256 x 1024."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads import config, generators
    from workloads.configs import DECONV

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = config(4)
    kb = td.build_kernels(s, mode="exact")
    rtrue = torch.from_numpy(generators.spikes(s.nz, s.nx, DECONV["n_spikes"], seed=0).astype(np.float32)).to(dev)
    clean = td.apply(kb, rtrue)
    sigma = float(torch.sqrt(torch.mean(clean.double() ** 2))) * 10.0 ** (-DECONV["snr_db"] / 20.0)
    noise = torch.from_numpy(generators.normal((s.nz, s.nx), seed=1).astype(np.float32)).to(dev)
    y = clean + sigma * noise
    lam, iters = DECONV["lam"], DECONV["iters"]
    eta = td.step_size(kb, lam, iters=300)
    r = torch.empty_like(y)
    w = torch.empty_like(y)
    ms = _events_ms(lambda: td.deconvolve(kb, y, lam, eta=eta, iters=iters, out=r, work=w), args.steps, args.warmup)
    err = float(torch.linalg.norm(r - rtrue) / torch.linalg.norm(rtrue))
    flops = iters * 2 * 2.0 * s.K * s.nz * s.nx
    # the same solve on a batch of 16 maps (16 noise draws of the same
    # reflectivity) in one call: one map fills only 16 workgroups of the tile
    nb = 16
    yb = torch.stack([clean + sigma * torch.from_numpy(generators.normal((s.nz, s.nx), seed=10 + b)
                                                      .astype(np.float32)).to(dev) for b in range(nb)])
    rb, wb = torch.empty_like(yb), torch.empty_like(yb)
    ms_b = _events_ms(lambda: td.deconvolve(kb, yb, lam, eta=eta, iters=iters, out=rb, work=wb), args.steps,
                      args.warmup)
    out = {
        "metric": "Tikhonov deconvolution, 200 gradient iterations through the line model (ms per solve)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (500 N(0,1) spikes, 40 dB Gaussian noise)",
        "config": {"workload": "256 x 1024 map, 65-tap exact kernels of the 64-element array, lambda 1e-3",
                   "iterations": iters, "eta": eta},
        "us_per_iteration": ms * 1e3 / iters, "achieved_tflops": flops / (ms * 1e-3) / 1e12,
        "rel_error_to_truth": err,
        "batch_of_16_maps": {"ms_per_solve_of_all": ms_b, "maps_per_s": nb / (ms_b * 1e-3),
                             "achieved_tflops": nb * flops / (ms_b * 1e-3) / 1e12},
    }
    print(json.dumps(out), flush=True)


def run_beamform(args):
    """Time-invariant beamformer from RF vs exact DAS: 64 speckle frames, 128 elements, 1024 x 256 px."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads import config, generators
    from workloads.configs import CYSTS, N_SCATTERERS

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = config(2)
    B, Z, X = args.batch, s.nz, s.nx
    rf = torch.empty((B, 1, s.n_elem, s.n_samples), device=dev, dtype=torch.float32)
    for b in range(B):
        x, z, a, _ = generators.speckle_with_cysts(N_SCATTERERS[2], s.field_w, s.field_d, CYSTS["n"], CYSTS["r_lo"],
                                                   CYSTS["r_hi"], seed=b)
        scat = torch.tensor(np.stack([x, z, a], 1), dtype=torch.float64, device=dev)
        td.simulate_rf(s, scat, out=rf[b])

    def refs_for(size):
        return np.minimum((np.arange(Z) // size) * size + size // 2, Z - 1).astype(np.int32)

    size = 64  # one receive law per 64 rows (3.75 mm)
    refs_h = refs_for(size)
    refs = torch.from_numpy(refs_h).to(dev)
    _, theta = td.build_kernels(s, mode="paper", ref_row=refs_h, with_theta=True)
    img = torch.empty((B, Z, X), device=dev, dtype=torch.float32)
    fd_ms = _events_ms(lambda: td.tidas_beamform(rf, s, ref_row=refs, theta=theta, out=img), args.steps, args.warmup)
    das_ms = _events_ms(lambda: td.das_beamform(rf, s, out=img), args.steps, args.warmup)
    # 2-D approximation error against DAS on frame 0, for several neighbourhood sizes
    d0 = td.das_beamform(rf[0], s)
    errors = {}
    for sz in (16, 64, 256):
        rh = refs_for(sz)
        _, th = td.build_kernels(s, mode="paper", ref_row=rh, with_theta=True)
        f0 = td.tidas_beamform(rf[0], s, ref_row=torch.from_numpy(rh).to(dev), theta=th)
        errors[f"law_per_{sz}_rows"] = float(torch.linalg.norm(f0 - d0) / torch.linalg.norm(d0))
    zs = s.z0 + np.arange(Z) * s.dz
    for depth in (25e-3, 35e-3):  # one law for the whole image (the paper's single reference curve)
        rh = np.full(Z, int(np.argmin(np.abs(zs - depth))), np.int32)
        _, th = td.build_kernels(s, mode="paper", ref_row=rh, with_theta=True)
        f0 = td.tidas_beamform(rf[0], s, ref_row=torch.from_numpy(rh).to(dev), theta=th)
        errors[f"one_law_at_{int(depth * 1e3)}mm"] = float(torch.linalg.norm(f0 - d0) / torch.linalg.norm(d0))
    out = {
        "metric": "frames/s, time-invariant beamformer from RF vs exact DAS (256x1024 px, 128 ch)",
        "value": B / (fd_ms * 1e-3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fd_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (speckle phantoms with cysts, RF synthesised on the GPU)",
        "config": {"workload": f"{B} frames, 128-ch plane wave, 256x1024 px, one receive law per {size} rows, "
                               "theta from paper mode", "global_batch": B},
        "das": {"frames_per_s": B / (das_ms * 1e-3), "ms_per_step": das_ms},
        "speedup_vs_das": das_ms / fd_ms,
        "rel_l2_vs_das_2d": errors,
    }
    if not (args.no_parity and args.no_cpu_baseline):
        from oracle import das as o_das, simulate as o_sim
        xs = s.x0 + np.arange(X) * s.dx
        okw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
                   n_samples=s.n_samples, angles=list(s.angles))
        dkw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, angles=list(s.angles), fnumber=s.fnumber)
        # a lighter phantom of the same kind for the oracle (2000 scatterers, cysts, seed 0)
        x, z, a, _ = generators.speckle_with_cysts(2000, s.field_w, s.field_d, CYSTS["n"], CYSTS["r_lo"],
                                                   CYSTS["r_hi"], seed=0)
        rf_o = o_sim.to_fp32(o_sim.simulate_rf(x, z, a, **okw))
        th_h = theta.cpu().numpy()
        if not args.no_parity:
            f_gpu = td.tidas_beamform(torch.from_numpy(rf_o).to(dev), s, ref_row=refs, theta=theta).cpu().numpy()
            f_ref = o_das.fixed_delay_das(rf_o, xs, zs, refs_h, **dkw, theta=th_h)
            out["rel_l2_vs_fp64"] = float(np.linalg.norm(f_gpu - f_ref) / np.linalg.norm(f_ref))
            out["parity_sample"] = "one 1024 x 256 frame of a 2000-scatterer phantom (oracle RF)"
        if not args.no_cpu_baseline:
            t_c = time.perf_counter()
            n_fr = 0
            while n_fr < 1 or time.perf_counter() - t_c < 5.0:
                o_das.fixed_delay_das(rf_o, xs, zs, refs_h, **dkw, theta=th_h)
                n_fr += 1
            out["cpu_baseline"] = {"value": n_fr / (time.perf_counter() - t_c), "unit": "frames/s", "cores": 1,
                                   "kind": "oracle",
                                   "sample": f"FP64 oracle fixed-delay beamformer on {n_fr} frames, about 5 s"}
    print(json.dumps(out), flush=True)


def run_separable(args):
    """Depth pass + lateral pass on 64 speckle maps of 1024 x 256: time, roofline, 2-D error against DAS."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads import config, generators
    from workloads.configs import CYSTS, N_SCATTERERS

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = config(2)
    B, Z, X, K = args.batch, s.nz, s.nx, s.K
    KX = 33
    R = torch.empty((B, Z, X), device=dev, dtype=torch.float32)
    phantoms = []
    for b in range(B):
        x, z, a, _ = generators.speckle_with_cysts(N_SCATTERERS[2], s.field_w, s.field_d, CYSTS["n"], CYSTS["r_lo"],
                                                   CYSTS["r_hi"], seed=b)
        phantoms.append((x, z, a))
        i, j, _, _ = generators.snap_to_grid(x, z, s.x0, s.dx, X, s.z0, s.dz, Z)
        R[b] = torch.from_numpy(generators.reflectivity_map(i, j, a, Z, X).astype(np.float32))
    kz = td.build_kernels(s, mode="exact")
    prep = td.prepare(kz)
    kx = td.build_kernels(s, K=KX, mode="lateral")
    Y1 = torch.empty_like(R)
    Y2 = torch.empty_like(R)
    td.apply(prep, R, out=Y1)
    lat_ms = _events_ms(lambda: td.apply_lateral(kx, Y1, out=Y2), args.steps, args.warmup)
    both_ms = _events_ms(lambda: (td.apply(prep, R, out=Y1), td.apply_lateral(kx, Y1, out=Y2)), args.steps,
                         args.warmup)
    lat_bytes = 8.0 * B * Z * X + 4.0 * Z * KX
    lat_gbs = lat_bytes / (lat_ms * 1e-3) / 1e9
    # 2-D error against DAS on frame 0 (phantom snapped to the grid, RF of the snapped scatterers)
    x, z, a = phantoms[0]
    _, _, zs_, xs_ = generators.snap_to_grid(x, z, s.x0, s.dx, X, s.z0, s.dz, Z)
    scat = torch.tensor(np.stack([xs_, zs_, a], 1), dtype=torch.float64, device=dev)
    d0 = td.das_beamform(td.simulate_rf(s, scat), s)
    y1 = td.apply(prep, R[0])
    nd = torch.linalg.norm(d0)
    errors = {"depth_pass_only": float(torch.linalg.norm(y1 - d0) / nd)}
    for kxn in (17, 33, 65):
        kk = td.build_kernels(s, K=kxn, mode="lateral")
        errors[f"with_lateral_{kxn}_taps"] = float(torch.linalg.norm(td.apply_lateral(kk, y1) - d0) / nd)
    out = {
        "metric": "frames/s, separable 2-D model (depth pass + lateral pass) at 256x1024 px",
        "value": B / (both_ms * 1e-3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": both_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (speckle phantoms with cysts snapped to the grid)",
        "config": {"workload": f"{B} frames of 1024 x 256 px, 129-tap exact depth kernels, {KX}-tap lateral kernels",
                   "global_batch": B},
        "lateral_pass": {"ms_per_step": lat_ms, "frames_per_s": B / (lat_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": lat_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": lat_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(B, LATERAL_TRAFFIC_FILE),
                     "kernel": "lateral_pass_kernel",
                     "bytes_per_launch": lat_bytes},
        "rel_l2_vs_das_2d": errors,
    }
    if not (args.no_parity and args.no_cpu_baseline):
        from oracle import kernels as o_k, tidas as o_t
        zs = s.z0 + np.arange(Z) * s.dz
        okw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
                   n_samples=s.n_samples, angles=list(s.angles), fnumber=s.fnumber)
        kz_o = o_k.exact_kernels(zs, s.dz, K, **okw)
        kx_o = o_k.lateral_kernels(zs, s.dx, KX, **okw)
        x, z, a = phantoms[0]
        i, j, _, _ = generators.snap_to_grid(x, z, s.x0, s.dx, X, s.z0, s.dz, Z)
        R_host = generators.reflectivity_map(i, j, a, Z, X).astype(np.float32)
        t_c = time.perf_counter()
        y_ref = o_t.apply_lateral(kx_o, o_t.apply(kz_o, R_host))
        cpu_s = time.perf_counter() - t_c
        if not args.no_parity:
            assert torch.equal(R[0].cpu(), torch.from_numpy(R_host))
            y_gpu = Y2[0].cpu().numpy()
            out["rel_l2_vs_fp64"] = float(np.linalg.norm(y_gpu - y_ref) / np.linalg.norm(y_ref))
            out["parity_sample"] = "frame 0 of the timed launch (kernels built by each side)"
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": 1.0 / cpu_s, "unit": "frames/s", "cores": 1, "kind": "oracle",
                                   "sample": "FP64 oracle depth + lateral pass on one frame"}
    print(json.dumps(out), flush=True)


def run_kgrad(args):
    """Gradient of the line model in its kernels: B frames of 1024 x 256, 129 taps."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads import config, generators

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = config(2)
    B, Z, X, K = args.batch, s.nz, s.nx, s.K
    R = generators.normal((B, Z, X), seed=0).astype(np.float32)
    Yb = generators.normal((B, Z, X), seed=1).astype(np.float32)
    Rd, Yd = torch.from_numpy(R).to(dev), torch.from_numpy(Yb).to(dev)
    G = torch.empty((Z, K), device=dev, dtype=torch.float32)
    ms = _events_ms(lambda: td.kernel_grad(Rd, Yd, K, out=G), args.steps, args.warmup)
    flops = 2.0 * B * Z * X * K
    tflops = flops / (ms * 1e-3) / 1e12
    out = {
        "metric": "kernel-gradient frames/s of the line model (1024 x 256 px, 129 taps) vs FP64 oracle",
        "value": B / (ms * 1e-3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (N(0,1) reflectivity maps and output gradients, seeded)",
        "config": {"workload": f"{B} frames of 1024 x 256 px, 129 taps (kernel gradient)", "global_batch": B},
        # the arithmetic is float32-level (split-bfloat16 parts, float32 sums, the
        # dropped cross terms below 2^-20 |ab|):
        # priced against the float32 matrix peak; the issued bf16 work (six
        # products per term, 160 source rows for 129 taps) beside it
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_MFMA_TFLOPS, "traffic": None, "flops_per_launch": flops,
                     "kernel": "kgrad_bf16_kernel + kgrad_reduce_kernel (whole call)",
                     "mfma_bf16_tflops_issued": 6.0 * flops * (32 * ((K + 62) // 32)) / K / (ms * 1e-3) / 1e12,
                     "mfma_bf16_frac": 6.0 * flops * (32 * ((K + 62) // 32)) / K / (ms * 1e-3) / 1e12
                     / BF16_MFMA_TFLOPS},
    }
    if not args.no_parity:
        # sampled entries against FP64 dot products over all frames and columns
        Gh = G.cpu().numpy()
        h = (K - 1) // 2
        rng = np.random.default_rng(2)
        got, want = [], []
        for _ in range(200):
            i, m = int(rng.integers(Z)), int(rng.integers(-h, h + 1))
            exp = (float(np.sum(Yb[:, i, :].astype(np.float64) * R[:, i - m, :].astype(np.float64)))
                   if 0 <= i - m < Z else 0.0)
            got.append(Gh[i, m + h])
            want.append(exp)
        got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
        out["rel_l2_vs_fp64"] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        out["parity_sample"] = "200 sampled (row, tap) entries of the timed launch"
    if not args.no_cpu_baseline:
        from oracle import tidas as o_t
        t_c = time.perf_counter()
        n_fr = 0
        while n_fr < 1 or time.perf_counter() - t_c < 5.0:
            o_t.kernel_grad(R[n_fr:n_fr + 1], Yb[n_fr:n_fr + 1], K)
            n_fr += 1
        out["cpu_baseline"] = {"value": n_fr / (time.perf_counter() - t_c), "unit": "frames/s", "cores": 1,
                               "kind": "oracle", "sample": f"FP64 oracle kernel gradient on {n_fr} frames, about 5 s"}
    print(json.dumps(out), flush=True)


def run_surrogate(args):
    """Train the kernel surrogate and compare surrogate-kernel tiDAS with exact-kernel tiDAS and DAS."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from paper_2507_15464_amd import surrogate as sg
    from workloads import config, generators
    from workloads.configs import CYSTS, N_SCATTERERS, SURROGATE

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s5 = config(5)
    K, Z, X = s5.K, s5.nz, s5.nx
    lo = (s5.z0, SURROGATE["fnumber"][0], np.radians(SURROGATE["angle_deg"][0]), SURROGATE["fc"][0])
    hi = (s5.z0 + (Z - 1) * s5.dz, SURROGATE["fnumber"][1], np.radians(SURROGATE["angle_deg"][1]),
          SURROGATE["fc"][1])

    def draws(n, seed):
        return torch.from_numpy(generators.kernel_params(n, lo[0], hi[0], SURROGATE["fnumber"], SURROGATE["angle_deg"],
                                                         SURROGATE["fc"], seed)).to(dev)

    # ---- data: exact normalised kernels generated on the GPU
    t0 = time.perf_counter()
    P_tr = draws(args.train_rows, 0)
    x_tr = sg.features(P_tr, lo, hi)
    t_tr, _ = sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, P_tr, K, normalise=True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    log(f"{args.train_rows} training kernels in {gen_s:.2f}s")

    # ---- training
    model = sg.Surrogate()
    model.load_layers([(W, b) for W, b in generators.mlp_init(SURROGATE["widths"], 0)])
    B = SURROGATE["batch"]
    idx_all = torch.from_numpy(generators.batch_indices(args.train_rows, B, args.train_steps, seed=2).astype(np.int32))
    idx_all = idx_all.to(dev)
    batches = [idx_all[i] for i in range(args.train_steps)]
    first = float(model.train_step(x_tr, t_tr, idx=batches[0]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    final = model.fit(x_tr, t_tr, batches, total_steps=args.train_steps, log_every=max(1, args.train_steps // 10),
                      log=lambda st, l: log(f"step {st} loss {l:.3e}"))
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    macs = sum(a * b for a, b in zip(SURROGATE["widths"][:-1], SURROGATE["widths"][1:]))
    train_flops = args.train_steps * B * 2.0 * macs * 3.0

    # ---- held-out kernels
    P_te = draws(4096, 1)
    ex_te, s_te = sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, P_te, K)
    pr_te = model.forward(sg.features(P_te, lo, hi), scale=s_te)
    heldout = sg.rel_l2(pr_te, ex_te)

    # ---- the 512 x 2048 image: rows at F# 1.5, 0 deg, 7.5 MHz
    zs = s5.z0 + np.arange(Z) * s5.dz
    P_img = torch.from_numpy(np.stack([zs, np.full(Z, 1.5), np.zeros(Z), np.full(Z, 7.5e6)], 1)).to(dev)
    bank_s, info = model.kernel_bank(s5, P_img, lo, hi, judge_rows=32, tol=1.0)
    bank_e, _ = sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, P_img, K)
    bank_err = sg.rel_l2(bank_s, bank_e)
    t_sur = _events_ms(lambda: model.forward(sg.features(P_img, lo, hi), scale=sg.aperture_scale(s5, P_img)), 20, 3)
    t_ex = _events_ms(lambda: sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, P_img, K), 20, 3)

    x, z, a, _ = generators.speckle_with_cysts(N_SCATTERERS[2], s5.field_w, s5.field_d, CYSTS["n"], CYSTS["r_lo"],
                                               CYSTS["r_hi"], seed=0)
    i, j, zsn, xsn = generators.snap_to_grid(x, z, s5.x0, s5.dx, X, s5.z0, s5.dz, Z)
    R = torch.from_numpy(generators.reflectivity_map(i, j, a, Z, X).astype(np.float32)).to(dev)
    y_s = td.apply(bank_s, R)
    y_e = td.apply(bank_e, R)
    tidas_err = sg.rel_l2(y_s, y_e)
    img_setup = s5.replace(fnumber=1.5, fc=7.5e6, angles=(0.0,))
    rf = td.simulate_rf(img_setup, torch.tensor(np.stack([xsn, zsn, a], 1), dtype=torch.float64, device=dev))
    d = td.das_beamform(rf, img_setup)
    approx_e, approx_s = sg.rel_l2(y_e, d), sg.rel_l2(y_s, d)

    # ---- the part of the exact kernels that changes within one RF sample of
    # depth: exact kernels of scatterers shifted by sub-sample offsets
    # (16 offsets spanning one two-way sample, c / (2 fs)) averaged, then the
    # exact bank's distance to that average.  Linear interpolation of the
    # channel data makes each kernel depend on the sub-sample phases of its
    # echoes; no function that is smooth on the scale of a sample can follow
    # that component, so it bounds a smooth surrogate's error from below.
    dzf = s5.c / (2.0 * s5.fs)
    avg = torch.zeros_like(bank_e)
    n_off = 16
    for k in range(n_off):
        Pk = P_img.clone()
        Pk[:, 0] += ((k + 0.5) / n_off - 0.5) * dzf
        ek, _ = sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, Pk, K)
        avg += ek / n_off
    phase_component = sg.rel_l2(avg, bank_e)
    surrogate_vs_phase_avg = sg.rel_l2(bank_s, avg)

    # ---- the paper's own cheap strategy on held-out configurations: paper-mode
    # banks from 1, 16 and 64 reference profiles; errors and build times
    held = [(1.5, 0.0, 7.5e6), (2.3, -7.0, 4.2e6), (1.2, 11.0, 9.1e6)]
    paper_cmp = []
    for fnum, adeg, fc in held:
        Pc = torch.from_numpy(np.stack([zs, np.full(Z, fnum), np.full(Z, np.radians(adeg)), np.full(Z, fc)], 1)).to(dev)
        ex_c, sc = sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, Pc, K)
        net_c = model.forward(sg.features(Pc, lo, hi), scale=sc)
        setup_c = s5.replace(fnumber=fnum, fc=fc, angles=(float(np.radians(adeg)),))
        rec = {"fnumber": fnum, "angle_deg": adeg, "fc_mhz": fc / 1e6, "surrogate_rel_l2": sg.rel_l2(net_c, ex_c),
               "surrogate_ms": _events_ms(lambda: model.forward(sg.features(Pc, lo, hi),
                                                                scale=sg.aperture_scale(s5, Pc)), 10, 2),
               "exact_ms": _events_ms(lambda: sg.kernels_at(s5, s5.fs, s5.t0, s5.cycles, s5.n_samples, s5.dz, Pc, K),
                                      10, 2)}
        for per, name in ((Z, "1"), (128, "16"), (32, "64")):
            refs = np.minimum((np.arange(Z) // per) * per + per // 2, Z - 1)
            kp = td.build_kernels(setup_c, K=K, mode="paper", ref_row=refs)
            rec[f"paper_{name}_profiles_rel_l2"] = sg.rel_l2(kp, ex_c)
            t0p = time.perf_counter()
            for _ in range(5):
                td.build_kernels(setup_c, K=K, mode="paper", ref_row=refs)
            torch.cuda.synchronize()
            rec[f"paper_{name}_profiles_ms"] = (time.perf_counter() - t0p) / 5 * 1e3
        paper_cmp.append(rec)
        log(f"held-out {rec}")

    # ---- throughput: 64 frames per launch on the surrogate bank, prepared
    # once (the bank is per geometry, like its conversion)
    nb = 64
    Rb = R.unsqueeze(0).repeat(nb, 1, 1).contiguous()
    Yb = torch.empty_like(Rb)
    prep_s = td.prepare(bank_s)
    app_ms = _events_ms(lambda: td.apply(prep_s, Rb, out=Yb), args.steps, args.warmup)
    hbm = (8.0 * Z * X * nb + 4.0 * Z * K) / (app_ms * 1e-3) / 1e9
    tflops = 2.0 * K * Z * X * nb / (app_ms * 1e-3) / 1e12
    out = {
        "metric": "surrogate-kernel tiDAS vs exact-kernel tiDAS (512x2048 px, 129 taps): rel-L2 and frames/s",
        "value": nb / (app_ms * 1e-3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": app_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MLP / f32 line model", "data": "synthetic (exact DAS kernels of random draws; speckle)",
        "config": {"workload": "MLP 4-256-256-256-129 GELU, 200k kernels, batch 1024; 512x2048 image",
                   "train_rows": args.train_rows, "train_steps": args.train_steps},
        "training": {"data_gen_s": gen_s, "ms": train_ms, "steps_per_s": args.train_steps / (train_ms * 1e-3),
                     "achieved_tflops_bf16": train_flops / (train_ms * 1e-3) / 1e12, "loss_first": first,
                     "loss_final": final},
        "heldout_kernel_rel_l2": heldout,
        "image": {"bank_rel_l2": bank_err, "judge": info, "surrogate_vs_exact_tidas_rel_l2": tidas_err,
                  "exact_tidas_vs_das_rel_l2": approx_e, "surrogate_tidas_vs_das_rel_l2": approx_s,
                  "sub_sample_phase_component_rel_l2": phase_component,
                  "surrogate_vs_phase_averaged_bank_rel_l2": surrogate_vs_phase_avg},
        "paper_mode_comparison": paper_cmp,
        "bank_generation_ms": {"surrogate": t_sur, "exact": t_ex, "speedup": t_ex / t_sur},
        "per_frame_with_bank_ms": {"surrogate": t_sur + app_ms / nb, "exact": t_ex + app_ms / nb},
        "line_model": {"tflops": tflops, "hbm_gbs_algorithmic": hbm, "hbm_frac": hbm / HBM_PEAK_GBS,
                       "frames_per_launch": nb, "kernel": td.line_kernel(K, nb, Z, X)},
    }
    print(json.dumps(out), flush=True)


def line_errors(setup, K, dev):
    """Paper-style 1-D error of the line model against DAS on the centre line.

    Single scatterers: the DAS response of a unit scatterer at row s along the
    whole line is the exact-mode kernel of row s with 2 Z - 1 taps; the line
    model's response is column s of its banded matrix.  Local error: squared
    relative l2 error inside the pulse's two-way envelope FWHM around the
    scatterer; global: over the whole line.  Line phantoms: on-grid on-axis
    scatterers, RF synthesised and beamformed by DAS on the x = 0 column."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    Z = setup.nz
    line = setup.replace(nx=1, x0=0.0)
    zs = setup.z0 + np.arange(Z) * setup.dz
    big = td.build_kernels(line, K=2 * Z - 1, mode="exact").cpu().numpy().astype(np.float64)
    H = Z - 1
    das_cols = np.stack([big[s, H - s:H - s + Z] for s in range(Z)], 1)  # [i][s]: DAS at row i of scatterer s
    w_fwhm = setup.cycles / setup.fc * setup.c / 2.0
    local_mask = np.abs(zs[:, None] - zs[None, :]) <= 0.5 * w_fwhm
    r25, r35 = int(np.argmin(np.abs(zs - 25e-3))), int(np.argmin(np.abs(zs - 35e-3)))
    banks = {"exact": td.build_kernels(line, K=K, mode="exact"),
             "paper_ref25mm": td.build_kernels(line, K=K, mode="paper", ref_row=[r25] * Z),
             "paper_ref35mm": td.build_kernels(line, K=K, mode="paper", ref_row=[r35] * Z),
             "line_ref25mm": td.build_kernels(line, K=K, mode="line", ref_row=[r25] * Z),
             "line_own_rows": td.build_kernels(line, K=K, mode="line")}
    # line phantoms (on-grid, on-axis), DAS from synthesised RF
    rows5 = np.linspace(0.15 * Z, 0.85 * Z, 5).round().astype(int)
    rng = np.random.default_rng(0)
    rows100 = np.sort(rng.choice(np.arange(int(0.05 * Z), int(0.95 * Z)), 100, replace=False))
    phantoms = {"5_uniform": (rows5, np.ones(5)), "5_rising": (rows5, np.linspace(0.5, 2.0, 5)),
                "100_uniform": (rows100, np.ones(100))}
    out = {}
    for name, kb in banks.items():
        M = np.zeros((Z, Z))
        kbn = kb.cpu().numpy().astype(np.float64)
        h = (K - 1) // 2
        for s in range(Z):
            lo_i, hi_i = max(0, s - h), min(Z, s + h + 1)
            for i in range(lo_i, hi_i):
                M[i, s] = kbn[i, i - s + h]
        d2 = das_cols ** 2
        e2 = (M - das_cols) ** 2
        valid = d2.sum(0) > 0
        glob = e2.sum(0)[valid] / d2.sum(0)[valid]
        loc_num = (e2 * local_mask).sum(0)
        loc_den = (d2 * local_mask).sum(0)
        okl = loc_den > 0
        loc = loc_num[okl] / loc_den[okl]
        rec = {"single_local_sq_median": float(np.median(loc)), "single_local_sq_mean": float(np.mean(loc)),
               "single_local_below_5pct": float(np.mean(loc < 0.05)),
               "single_global_sq_median": float(np.median(glob)), "single_global_below_5pct": float(np.mean(glob < 0.05))}
        for pname, (rows, amp) in phantoms.items():
            scat = torch.tensor(np.stack([np.zeros(rows.size), zs[rows], amp], 1), dtype=torch.float64, device=dev)
            rf = td.simulate_rf(line, scat)
            d = td.das_beamform(rf, line).cpu().numpy()[:, 0].astype(np.float64)
            Rm = np.zeros((Z, 1), np.float32)
            Rm[rows, 0] = amp
            y = td.apply(kb, torch.from_numpy(Rm).to(dev)).cpu().numpy()[:, 0].astype(np.float64)
            near = np.zeros(Z, bool)
            for r in rows:
                near |= np.abs(zs - zs[r]) <= 0.5 * w_fwhm
            rec[pname] = {"global_sq": float(np.sum((y - d) ** 2) / np.sum(d ** 2)),
                          "local_sq": float(np.sum(((y - d) ** 2)[near]) / np.sum((d ** 2)[near])),
                          "rel_l2": float(np.linalg.norm(y - d) / np.linalg.norm(d))}
        out[name] = rec
    return out


def run_approx(args):
    import torch

    from workloads import config

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    res = {}
    for k in (1, 2):
        s = config(k)
        t0 = time.perf_counter()
        res[f"config{k}"] = line_errors(s, s.K, dev)
        log(f"config {k}: {time.perf_counter() - t0:.1f}s")
    out = {"metric": "paper-style 1-D tiDAS-vs-DAS squared error (on-axis line, plane wave)",
           "value": res["config2"]["exact"]["single_local_sq_median"], "unit": "squared rel. error (median, local)",
           "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic on-axis scatterers", "config": {"workload": "configs 1 and 2 geometry, x = 0 column"},
           "errors": res, "paper_threshold": 0.05}
    print(json.dumps(out), flush=True)


def run_study(args):
    """The single-point study for every (centre frequency, focal depth) of the
    workload; sampled pairs of one setting against the oracle."""
    import numpy as np
    import torch

    import paper_2507_15464_amd as td
    from workloads.configs import STUDY, study_focal_index, study_line_half, study_setup

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    settings = []
    parity = None
    cpu = None
    for fc in STUDY["fcs"]:
        s = study_setup(fc)
        P = s.nz
        Ql = study_line_half(s)
        Qh = min(511, 4 * int(np.ceil(8 * s.sigma * s.fs)))
        for zf in STUDY["foci"]:
            f = study_focal_index(s, zf)
            n_tx = td.kossoff_tx_count(s, s.z0 + f * s.dz, STUDY["kossoff"])
            run = lambda: td.point_study(s, n_tx, P, s.z0, s.dz, f, Ql, stats_half=Qh)  # noqa: E731
            ms = _events_ms(run, 1, 1)
            out = run()
            torch.cuda.synchronize()
            th = out["theta"].cpu().numpy()
            lo = out["err_local"].cpu().numpy()
            gl = out["err_global"].cpu().numpy()
            st = out["stats"].cpu().numpy()
            d_fwhm = np.abs(st[:, 3] - st[:, 2])
            q = lambda v: [float(x) for x in np.percentile(v, [25, 50, 75])]  # noqa: E731
            rec = {"fc_mhz": fc / 1e6, "focus_mm": (s.z0 + f * s.dz) * 1e3, "focal_index": f, "n_tx": n_tx,
                   "window_mm": out["window"].item() * 1e3, "ms": ms, "pairs_per_s": P * P / (ms * 1e-3),
                   "local_below_5pct": float(np.mean(lo < 0.05)), "global_below_5pct": float(np.mean(gl < 0.05)),
                   "curves_covering_all_points_local_5pct": int(np.sum(np.all(lo < 0.05, axis=1))),
                   "focal_curve_local_below_5pct": float(np.mean(lo[f] < 0.05)),
                   "theta_range": [float(th.min()), float(th.max())],
                   "theta_diag_range": [float(np.diag(th).min()), float(np.diag(th).max())],
                   "abs_dfwhm_um_quartiles": [1e6 * v for v in q(d_fwhm)],
                   "peak_ratio_tidas_over_das_quartiles": q(st[:, 1] / st[:, 0]),
                   "das_peak_over_focal_peak_range": [float((st[:, 0] / st[f, 0]).min()),
                                                      float((st[:, 0] / st[f, 0]).max())]}
            settings.append(rec)
            log(f"study fc {fc / 1e6} MHz focus {rec['focus_mm']:.2f} mm: {ms:.1f} ms, "
                f"local<5% {rec['local_below_5pct']:.3f}")
            if parity is None and not args.no_parity:
                from oracle import point_study as ps
                o = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
                         n_samples=s.n_samples, fnumber=s.fnumber, n_tx=n_tx)
                pts, refs = [0, f, P // 2, P - 1], [0, f, P - 1]
                t0 = time.perf_counter()
                tho, loo, glo, W, _ = ps.study(o, P, s.z0, s.dz, f, Ql, refs=refs, points=pts)
                cpu_s = time.perf_counter() - t0
                sub = np.ix_(refs, pts)
                parity = {"pairs": len(refs) * len(pts), "setting": f"{fc / 1e6} MHz, focus {zf * 1e3:.0f} mm",
                          "theta_max_rel": float(np.max(np.abs(th[sub] - tho) / np.abs(tho))),
                          "err_local_max_abs": float(np.max(np.abs(lo[sub] - loo))),
                          "err_global_max_abs": float(np.max(np.abs(gl[sub] - glo))),
                          "window_rel": abs(out["window"].item() - W) / W}
                if not args.no_cpu_baseline:
                    # the oracle's time per pair (an echo per point, lines per pair)
                    cpu = {"value": len(refs) * len(pts) / cpu_s, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                           "sample": f"{len(refs)} x {len(pts)} pairs of the {P}-point study"}
    total_ms = sum(r["ms"] for r in settings)
    pairs = len(settings) * STUDY["n_points"] ** 2
    out = {"metric": "single-point study (Sec. 3.1-3.3): (delay curve, scatterer) pairs per second",
           "value": pairs / (total_ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (unit scatterers on the probe axis)",
           "config": {"workload": "192 elements, 0.3 mm pitch, 50 MHz, F/1, 600 points 2-42 mm, focused transmit "
                                  "with a Kossoff aperture, 4 frequencies x 3 focal depths"},
           "settings": settings, "parity": parity, "cpu_baseline": cpu, "paper_threshold": 0.05}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
