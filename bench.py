#!/usr/bin/env python3
"""Benchmark of the known-operator CT hot path on one MI355X.

One step = the whole path over one synthetic 512^3 cone-beam workload
(12 seeded random ellipsoids at 0.5 mm, 360 views over 360 deg, 1024 x 768
detector at 0.8 mm, SID 750 mm, SDD 1200 mm), resident in HBM:

    forward projection  vol -> proj                 (ph_project_cone3d)
    weighting + Ram-Lak row filter  proj -> q       (ph_weight_filter_3d)
    back-projection  q -> vol_rec                   (ph_backproject_cone3d)

The last two are exactly ph_fdk_cone3d, called as its two stages so that each
kernel is timed with HIP events on the stream it runs on.  The JSON line
reports back-projection GUPS (voxel-view updates per second of the FDK
stage), forward-projection Gsamples/s, a roofline entry for the dominant
kernel and for each kernel, and the FP64 oracle timed on a bounded sample on
the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X figures: 256 CUs at 2.4 GHz, 64 FP32 lanes per CU per clock without
# packed math; HBM3E 8 TB/s.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 39.3 T lane-ops/s
PEAK_HBM_GBS = 8000.0
# Algorithmic lane-ops per unit of work: the operations the interpolation itself needs.
OPS_PER_UPDATE = 11.0      # back-projection: v coordinate, floor/fract, 3 lerps, accumulate
OPS_PER_SAMPLE = 26.0      # forward projection: 3 coordinates, 3 floor/fract, 7 lerps, accumulate

# HBM bytes per launch at 512^3 from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by
# what the same counter reads for a plain 1 GiB device-to-device copy (FETCH_SIZE 524315 KiB, WRITE_SIZE 1048576 KiB).
# A record holds for the kernel's device sources it was taken on (hash below); after any change to them the traffic
# is reported as null.
COPY_BYTES = 1 << 30
COPY_FETCH_KIB, COPY_WRITE_KIB = 524315.0, 1048576.0
MEASURED_TRAFFIC = {
    "fp_cone": {"fetch_kib": 6.47788e+07, "write_kib": 1.24095e+06,
             "sources": ('cone_fp.hip', 'device_util.h'), "sha256_16": "3689f3d998d3b903"},
    "bp_cone": {"fetch_kib": 8.80846e+06, "write_kib": 524288,
             "sources": ('cone_bp.hip', 'device_util.h'), "sha256_16": "e1f54f92b2136414"},
    "weight_filter": {"fetch_kib": 563800, "write_kib": 1.10592e+06,
                   "sources": ('filter.hip', 'fft.h'), "sha256_16": "89a6c98d7d5f61cc"},
    "fpT_cone": {"fetch_kib": 8.37076e+06, "write_kib": 524288,
              "sources": ('adjoint.hip', 'device_util.h'), "sha256_16": "d6d2b86b350f2a7c"},
    "bpT_cone": {"fetch_kib": 2.75112e+06, "write_kib": 2.27029e+07,
              "sources": ('cone_bp.hip', 'device_util.h'), "sha256_16": "e1f54f92b2136414"},
}


def add_hbm(kv, alg_bytes):
    """HBM view of a VALU-bound kernel, beside its VALU roofline: algorithmic
    bytes (inputs read once, outputs written once) and, where counters are on
    record, the measured HBM bytes, each per launch time and as a fraction of
    the 8 TB/s peak."""
    s = kv["ms"] * 1e-3
    kv["hbm"] = {"algorithmic_bytes": alg_bytes, "algorithmic_GBps": alg_bytes / s / 1e9,
                 "algorithmic_frac": alg_bytes / s / 1e9 / PEAK_HBM_GBS,
                 "measured_GBps": None if kv.get("traffic") is None else kv["traffic"] / s / 1e9,
                 "measured_frac": None if kv.get("traffic") is None else kv["traffic"] / s / 1e9 / PEAK_HBM_GBS}


def measured_traffic(name):
    """HBM bytes per launch of kernel `name`, or None if its sources changed since the counters were taken."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(name)
    if rec is None:
        return None
    m = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_1904_13342_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    if m.hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["fetch_kib"] * COPY_BYTES / COPY_FETCH_KIB + rec["write_kib"] * COPY_BYTES / COPY_WRITE_KIB


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cone3d_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--workload", choices=("fdk", "adjoint", "corrector", "tv", "filter2d", "fan2d", "precision",
                                           "copyref"),
                    default="fdk",
                    help="fdk: the projector / FDK hot path (default); adjoint: the 512^3 operators as differentiable "
                         "layers, forward and matched backward (A, A^T, B, B^T); "
                         "corrector: the learned-corrector training run; "
                         "tv: sparse-view TV-regularised iterative reconstruction; "
                         "filter2d: learning the 2D reconstruction filter alone from the ramp; "
                         "precision: FP16 / BF16 storage against FP32 at 512^3 (RMSE and speed); "
                         "copyref: one plain 1 GiB device copy, the reference that scales the HBM byte counters")
    ap.add_argument("--iters", type=int, default=500, help="tv: iterations")
    ap.add_argument("--lam", type=float, default=3e-3, help="tv: TV weight")
    ap.add_argument("--train-steps", type=int, default=2000, help="corrector: Adam steps")
    ap.add_argument("--batch", type=int, default=16, help="corrector: training phantoms per step")
    ap.add_argument("--sigma", type=float, default=0.01, help="corrector: Gaussian noise on the line integrals")
    ap.add_argument("--lr", type=float, default=1e-3, help="corrector: Adam learning rate")
    ap.add_argument("--taps", type=int, default=1024, help="corrector: filter length M")
    ap.add_argument("--k-init", choices=("ramp", "ramlak"), default="ramp",
                    help="corrector: initial filter (the ramp, or Ram-Lak sampled on the M-point grid)")
    ap.add_argument("--w-unit", type=float, default=1e-2,
                    help="corrector: unit W is learned in (W moves by about lr * w_unit per step)")
    ap.add_argument("--save", default=None, help="corrector: write the learned K, W and losses to this .npz")
    return ap.parse_args()


def count_samples(spec, device):
    """Number of ray samples inside the open index box (-1, N)^3: for every
    ray, the integers k strictly between the entry and exit parameters of
    the line a + k*step*d through that box (a = point of the ray closest to
    the isocentre, d unit direction).  Computed in float64 with torch."""
    import torch
    nz, ny, nx = spec.vol_shape
    sz, sy, sx = spec.vol_spacing
    oz, oy, ox = spec.origin
    nv, nu = spec.det_shape
    dv, du = spec.det_spacing
    u = (torch.arange(nu, dtype=torch.float64, device=device) - (nu - 1) / 2) * du
    v = (torch.arange(nv, dtype=torch.float64, device=device) - (nv - 1) / 2) * dv
    V, U = torch.meshgrid(v, u, indexing="ij")
    total = 0
    for k in range(spec.n_proj):
        b = spec.angular_range * k / spec.n_proj
        c = (math.cos(b), math.sin(b))
        e = (-math.sin(b), math.cos(b))
        src = (-spec.sid * c[0], -spec.sid * c[1], 0.0)
        dx = spec.sdd * c[0] + U * e[0]
        dy = spec.sdd * c[1] + U * e[1]
        dz = V
        n = torch.sqrt(dx * dx + dy * dy + dz * dz)
        dx, dy, dz = dx / n, dy / n, dz / n
        t0 = -(src[0] * dx + src[1] * dy)
        lo = torch.full_like(U, -math.inf)
        hi = torch.full_like(U, math.inf)
        ok = torch.ones_like(U, dtype=torch.bool)
        for a, d, o, s, N in ((src[0], dx, ox, sx, nx), (src[1], dy, oy, sy, ny), (0.0, dz, oz, sz, nz)):
            p0 = (a + t0 * d - o) / s
            ee = spec.step * d / s
            nonzero = ee.abs() > 1e-300
            safe = torch.where(nonzero, ee, torch.ones_like(ee))
            t1 = (-1.0 - p0) / safe
            t2 = (N - p0) / safe
            lo = torch.where(nonzero, torch.maximum(lo, torch.minimum(t1, t2)), lo)
            hi = torch.where(nonzero, torch.minimum(hi, torch.maximum(t1, t2)), hi)
            ok &= nonzero | ((p0 > -1.0) & (p0 < N))
        cnt = torch.clamp(torch.ceil(hi) - torch.floor(lo) - 1.0, min=0.0)
        total += int(torch.where(ok & (hi > lo), cnt, torch.zeros_like(cnt)).sum().item())
    return total


def cpu_baseline(spec, vol_host, target_s):
    """The FP64 oracle on a bounded sample of the same workload: back-projection
    of a set of z slices (all views) and forward projection of a set of views.
    Rates are per second of wall time on all host cores."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    nz = spec.vol_shape[0]
    nvox_slice = spec.vol_shape[1] * spec.vol_shape[2]
    q = np.zeros((spec.n_proj,) + tuple(spec.det_shape))
    # calibrate on one slice, then size the sample to ~target_s/2 of back-projection
    t = time.perf_counter()
    oracle.backproject(spec, q, slices=[nz // 2])
    per_slice = max(time.perf_counter() - t, 1e-3)
    n_sl = int(max(1, min(nz, (0.5 * target_s) / per_slice)))
    slices = sorted(set(int(round(x)) for x in np.linspace(0, nz - 1, n_sl)))
    rng = np.random.default_rng(0)
    q = rng.standard_normal((spec.n_proj,) + tuple(spec.det_shape)).astype(np.float32).astype(np.float64)
    t = time.perf_counter()
    oracle.backproject(spec, q, slices=slices)
    t_bp = time.perf_counter() - t
    bp_gups = len(slices) * nvox_slice * spec.n_proj / t_bp / 1e9
    # forward projection: calibrate on one view, then ~target_s/2
    f = vol_host.astype(np.float64)
    t = time.perf_counter()
    oracle.project(spec, f, views=[0])
    per_view = max(time.perf_counter() - t, 1e-3)
    n_v = int(max(1, min(spec.n_proj, (0.5 * target_s) / per_view)))
    views = sorted(set(int(round(x)) for x in np.linspace(0, spec.n_proj - 1, n_v)))
    t = time.perf_counter()
    oracle.project(spec, f, views=views)
    t_fp = time.perf_counter() - t
    samples = oracle.count_samples(spec, views=views)
    return {
        "value": bp_gups,
        "unit": "GUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle back-projection of {len(slices)} of {nz} z-slices over all {spec.n_proj} views "
                   f"({t_bp:.1f} s) and forward projection of {len(views)} of {spec.n_proj} views ({t_fp:.1f} s)"),
        "fp_gsamples_per_s": samples / t_fp / 1e9,
    }


def corrector_main(args):
    """Learned-corrector training on the short-scan cone-beam workload (256^3 at
    1 mm, 248 views over 200 deg, 620 x 480 detector at 1 mm): training
    phantoms are seeds 0..batch-1, projected by the library's own projector;
    every step adds fresh Gaussian noise and takes one Adam step on K (M taps,
    ramp initialisation, learned in units of the ramp's bin step) and W (ones,
    learned in units of 1e-2).  Held-out seeds 1000-1003 (noise drawn
    once) give the RMSE of the learned reconstruction, of the ramp
    initialisation, of plain Ram-Lak / Parker FDK and of Ram-Lak sampled on
    the learned filter's grid, over the whole volume and over the covered
    cylinder (r <= 128 mm, |z| < 124 mm)."""
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config("cone3d_256_short")
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)

    def data(seeds):
        vols = torch.empty((len(seeds),) + tuple(spec.vol_shape), dtype=torch.float32, device=dev)
        for b, s in enumerate(seeds):
            prm = synth.random_ellipsoids(s, spec.n_figures, spec.vol_shape, spec.vol_spacing)
            vols[b] = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=2, device=dev,
                                                 dtype=torch.float32)
        return ph.project_cone3d(g, mats, vols), vols

    t0 = time.perf_counter()
    p_train, x_train = data(list(range(args.batch)))
    p_test, x_test = data([1000, 1001, 1002, 1003])
    gen = torch.Generator(device=dev).manual_seed(2024)
    p_test += args.sigma * torch.randn(p_test.shape, device=dev, generator=gen)
    torch.cuda.synchronize()
    print(f"[corrector] data ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    # inscribed cylinder (r <= 128 mm) over the slices every view covers (|z| < 124 mm)
    zs, ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    Zc = torch.as_tensor(zs, device=dev).view(-1, 1, 1)
    Yc = torch.as_tensor(ys, device=dev).view(1, -1, 1)
    Xc = torch.as_tensor(xs, device=dev).view(1, 1, -1)
    fov = ((Xc * Xc + Yc * Yc <= 128.0 ** 2) & (Zc.abs() < 124.0)).expand(tuple(spec.vol_shape))

    def rmse(x, region=None):
        d = (x.double() - x_test.double()) ** 2
        if region is not None:
            d = d[:, region]
        return float(d.mean().sqrt())

    tau = spec.det_spacing[1] * spec.sid / spec.sdd
    K0 = ph.filter_response(args.k_init, args.taps, tau) if args.k_init == "ramlak" else None
    corr = ph.LearnedCorrector(g, mats, M=args.taps, K=K0, lr=args.lr, w_unit=args.w_unit)
    x_init = corr.reconstruct(p_test)
    x_plain = ph.fdk_cone3d(g, mats, p_test)
    tau = spec.det_spacing[1] * spec.sid / spec.sdd
    x_rl = ph.fdk_cone3d(g, mats, p_test, K=ph.filter_response("ramlak", args.taps, tau).to(dev))
    rmse_init, rmse_plain, rmse_rl = rmse(x_init), rmse(x_plain), rmse(x_rl)
    fov_init, fov_plain, fov_rl = rmse(x_init, fov), rmse(x_plain, fov), rmse(x_rl, fov)
    del x_init, x_plain, x_rl
    noisy = torch.empty_like(p_train)
    noise = torch.empty_like(p_train)
    losses = []
    step_ms = []
    for k in range(args.train_steps):
        noise.normal_(generator=gen)
        torch.add(p_train, noise, alpha=args.sigma, out=noisy)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        loss = corr.step(noisy, x_train)
        e1.record()
        losses.append(loss)
        step_ms.append((e0, e1))
        if (k + 1) % 100 == 0 or k + 1 == args.train_steps:
            torch.cuda.synchronize()
            print(f"[corrector] step {k + 1}: loss {float(loss):.5e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in step_ms]
    losses = [float(v) for v in losses]
    x_learned = corr.reconstruct(p_test)
    rmse_learned, fov_learned = rmse(x_learned), rmse(x_learned, fov)
    line = {
        "metric": "learned-corrector training steps/s (FDK + MSE + B^T + K/W gradients + Adam)",
        "value": 1e3 / float(np.mean(ms[1:] if len(ms) > 1 else ms)),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.train_steps,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic: seeded random ellipsoids projected by the library's projector, Gaussian noise",
        "config": {"workload": f"cone3d 256^3 at 1 mm, {spec.n_proj} views over 200 deg, 620x480 detector at 1 mm",
                   "batch": args.batch, "taps": args.taps, "sigma": args.sigma, "lr": args.lr,
                   "K_init": args.k_init, "K_unit": corr.k_unit, "W_unit": corr.w_unit},
        "ms_per_step": float(np.mean(ms[1:] if len(ms) > 1 else ms)),
        "loss_first": losses[0],
        "loss_last10": float(np.mean(losses[-10:])),
        "rmse_heldout": {"learned": rmse_learned, "ramp_init": rmse_init, "plain_ramlak_parker_fdk": rmse_plain,
                         "ramlak_on_the_learned_grid": rmse_rl},
        "rmse_heldout_covered_cylinder": {"learned": fov_learned, "ramp_init": fov_init,
                                          "plain_ramlak_parker_fdk": fov_plain, "ramlak_on_the_learned_grid": fov_rl},
    }
    if args.save:
        np.savez(args.save, K=corr.K.cpu().numpy(), W=corr.W.cpu().numpy(), losses=np.array(losses),
                 step_ms=np.array(ms))
    print(json.dumps(line), flush=True)
    return corr


def tv_main(args):
    """Sparse-view TV-regularised iterative reconstruction (Sec. III.B.1): a
    256^2 image of 10 seeded random ellipses at 1 mm, 30 parallel views over
    180 deg, 363 bins at 1 mm, 2% additive Gaussian noise (sigma = 0.02 x the
    largest line integral), Adam from zero on mean((A x - p)^2) + lam TV(x).
    Reports iterations per second and the RMSE of the result (isotropic TV,
    and the anisotropic reading run the same way) and of FBP."""
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config("par2d_64").with_(vol_shape=(256, 256), det_shape=(363,), n_proj=30)
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    prm = synth.random_ellipses(spec.seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
    f = synth.rasterize_ellipses(prm, spec.vol_shape, spec.vol_spacing, sub=4).to(dev, torch.float32).contiguous()
    p = ph.project_par2d(g, rv, f)
    gen = torch.Generator(device=dev).manual_seed(30)
    p = (p + 0.02 * p.abs().max() * torch.randn(p.shape, device=dev, generator=gen)).contiguous()
    rmse = lambda x: float(((x.double() - f.double()) ** 2).mean().sqrt())
    rmse_fbp = rmse(ph.fbp_par2d(g, rv, p))
    it = ph.TVReconstruction("par2d", g, rv, p, lam=args.lam, eps=1e-2, lr=2e-2)
    it.run(10)   # warm-up iterations are part of the run
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    out = it.run(args.iters - 10)   # one library call: the loop runs inside the library
    e1.record()
    torch.cuda.synchronize()
    data, tvv = out[0], out[1]
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / (args.iters - 10)
    # the anisotropic reading of TV (sum of absolute differences), same weight and steps
    ia = ph.TVReconstruction("par2d", g, rv, p, lam=args.lam, eps=1e-2, lr=2e-2, anisotropic=True)
    e0.record()
    ia.run(args.iters)
    e1.record()
    torch.cuda.synchronize()
    ms_aniso = e0.elapsed_time(e1) / args.iters
    line = {
        "metric": "sparse-view TV iterative reconstruction iterations/s (A, residual, A^T, TV, Adam)",
        "value": 1e3 / ms,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.iters,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic: 10 seeded random ellipses, 2% Gaussian noise",
        "config": {"workload": "par2d 256x256 at 1 mm, 30 views over 180 deg, 363 bins at 1 mm",
                   "lam": args.lam, "eps": 1e-2, "lr": 2e-2},
        "ms_per_iteration": ms,
        "host_ms_per_iteration": wall * 1e3 / (args.iters - 10),
        "data_term_last": float(data),
        "tv_last": float(tvv),
        "rmse": {"tv": rmse(it.x), "tv_anisotropic": rmse(ia.x), "fbp": rmse_fbp},
        "ms_per_iteration_anisotropic": ms_aniso,
    }
    print(json.dumps(line), flush=True)


def count_samples_2d(spec, curved, device):
    """Ray samples of a 2D fan geometry inside the open index box (-1, N)^2,
    counted in float64 like count_samples (flat or equiangular detector)."""
    import torch
    ny, nx = spec.vol_shape
    sy, sx = spec.vol_spacing
    oy, ox = spec.origin
    nu, du = spec.det_shape[0], spec.det_spacing[0]
    u = (torch.arange(nu, dtype=torch.float64, device=device) - (nu - 1) / 2) * du
    total = 0
    for k in range(spec.n_proj):
        b = spec.angular_range * k / spec.n_proj
        c, e = (math.cos(b), math.sin(b)), (-math.sin(b), math.cos(b))
        src = (-spec.sid * c[0], -spec.sid * c[1])
        if curved:
            gam = u / spec.sdd
            dx, dy = torch.cos(gam) * c[0] + torch.sin(gam) * e[0], torch.cos(gam) * c[1] + torch.sin(gam) * e[1]
        else:
            dx, dy = spec.sdd * c[0] + u * e[0], spec.sdd * c[1] + u * e[1]
            n = torch.sqrt(dx * dx + dy * dy)
            dx, dy = dx / n, dy / n
        t0 = -(src[0] * dx + src[1] * dy)
        lo = torch.full_like(u, -math.inf)
        hi = torch.full_like(u, math.inf)
        for a, d, o, sp, N in ((src[0], dx, ox, sx, nx), (src[1], dy, oy, sy, ny)):
            p0 = (a + t0 * d - o) / sp
            ed = spec.step * d / sp
            t1, t2 = (-1.0 - p0) / ed, (N - p0) / ed
            lo = torch.maximum(lo, torch.minimum(t1, t2))
            hi = torch.minimum(hi, torch.maximum(t1, t2))
        n_in = torch.clamp(torch.ceil(hi) - torch.floor(lo) - 1, min=0)
        total += int(n_in.sum().item())
    return total


def fan2d_main(args):
    """The 2D fan-beam workload (512^2 at 0.5 mm of 10 seeded random ellipses,
    360 views over 360 deg, 725 bins of 1 mm, SID 750 mm, SDD 1200 mm) on the
    flat and on the equiangular (curved) detector: forward projection and
    FBP (weighting, filter, back-projection) timed with HIP events (median of
    five), and the FBP's RMSE against the phantom."""
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    out = {}
    for name, kind in (("flat", "fan2d"), ("curved", "fan2d_curved")):
        spec = synth.config("fan2d_512").with_(kind=kind)
        g = ph.from_spec(spec)
        rv = ph.ray_vectors_2d(g)
        prm = synth.random_ellipses(spec.seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_ellipses(prm, spec.vol_shape, spec.vol_spacing, sub=4).to(dev, torch.float32).contiguous()
        p = torch.empty((spec.n_proj, spec.det_shape[0]), dtype=torch.float32, device=dev)
        x = torch.empty_like(f)
        ws = torch.empty(ph.workspace_bytes_2d(g, 1), dtype=torch.uint8, device=dev)
        ph.fbp_fan2d(g, rv, ph.project_fan2d(g, rv, f, out=p), out=x, ws=ws)   # warm-up
        torch.cuda.synchronize()
        fp_ms, fbp_ms = [], []
        for _ in range(5):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            ph.project_fan2d(g, rv, f, out=p)
            ev[1].record()
            ph.fbp_fan2d(g, rv, p, out=x, ws=ws)
            ev[2].record()
            torch.cuda.synchronize()
            fp_ms.append(ev[0].elapsed_time(ev[1]))
            fbp_ms.append(ev[1].elapsed_time(ev[2]))
        fp_t, fbp_t = sorted(fp_ms)[2], sorted(fbp_ms)[2]
        samples = count_samples_2d(spec, name == "curved", dev)
        updates = spec.vol_shape[0] * spec.vol_shape[1] * spec.n_proj
        out[name] = {"fp_ms": fp_t, "fbp_ms": fbp_t, "fp_gsamples_per_s": samples / fp_t / 1e6,
                     "fbp_gups": updates / fbp_t / 1e6, "samples": samples,
                     "rmse_fbp": float(((x.double() - f.double()) ** 2).mean().sqrt())}
    line = {
        "metric": "2D fan-beam forward projection Gsamples/s and FBP GUPS, flat vs equiangular detector",
        "value": out["curved"]["fbp_gups"], "unit": "GUPS (FBP, curved detector)", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic: 10 seeded random ellipses",
        "config": {"workload": "fan2d 512x512 at 0.5 mm, 360 views over 360 deg, 725 bins at 1 mm "
                               "(flat pitch or arc length), SID 750, SDD 1200"},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def filter2d_main(args):
    """Learning the reconstruction filter alone (Sec. III.B, Eq. 6): 2D
    parallel beam, 256^2 at 1 mm, 360 views over 180 deg, 363 bins at 1 mm,
    batch 8 noise-free phantoms projected by the library's projector, K on
    the 1024-point grid initialised with the ramp, Adam.  Reports steps/s and
    the learned filter's distance to Ram-Lak over the lowest frequencies."""
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config("par2d_64").with_(vol_shape=(256, 256), det_shape=(363,), n_proj=360)
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    imgs = torch.stack([synth.rasterize_ellipses(synth.random_ellipses(s, spec.n_figures, spec.vol_shape,
                                                                       spec.vol_spacing),
                                                 spec.vol_shape, spec.vol_spacing, sub=4) for s in range(8)])
    imgs = imgs.to(dev, torch.float32).contiguous()
    sino = ph.project_par2d(g, rv, imgs)
    lf = ph.LearnedFilter2D(g, rv, lr=args.lr)
    rl = ph.filter_response("ramlak", lf.M, lf.tau).numpy().astype(np.float64)
    band = np.r_[0:16, lf.M - 15:lf.M]
    dist = lambda: float(np.linalg.norm(lf.K.cpu().numpy()[band] - rl[band]))
    d0 = dist()
    losses = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.train_steps):
        losses.append(lf.step(sino, imgs))
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.train_steps
    losses = [float(v) for v in losses]
    line = {
        "metric": "2D filter learning steps/s (FBP with K, MSE, B^T, dK, Adam)",
        "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.train_steps, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic: 8 seeded random-ellipse phantoms, noise-free projections",
        "config": {"workload": "par2d 256x256 at 1 mm, 360 views over 180 deg, 363 bins at 1 mm", "batch": 8,
                   "taps": lf.M, "lr": args.lr},
        "ms_per_step": ms, "loss_first": losses[0], "loss_last": losses[-1],
        "low_band_distance_to_ramlak": {"ramp_init": d0, "learned": dist()},
        "dc": {"learned": float(lf.K[0]), "ramlak": float(rl[0]), "ramp": 0.0},
    }
    if args.save:
        np.savez(args.save, K=lf.K.cpu().numpy(), ramlak=rl, losses=np.array(losses))
    print(json.dumps(line), flush=True)


def precision_main(args):
    """FP16 and BF16 storage against FP32 on the 512^3 workload: the phantom is
    stored in each type, forward projected and reconstructed by FDK in that
    type (FP32 arithmetic throughout), and each reconstruction's RMSE against
    the FP32 phantom is reported with the kernels' times (median of three
    repetitions into preallocated outputs)."""
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config("cone3d_512")
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    prm = synth.random_ellipsoids(spec.seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
    vol = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=1, device=dev,
                                     dtype=torch.float32).contiguous()
    # voxels inside the inscribed cylinder (radius 128 mm), which every view
    # covers over the full height at this magnification
    _, ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    Y = torch.as_tensor(ys, device=dev).view(-1, 1)
    X = torch.as_tensor(xs, device=dev).view(1, -1)
    mask = (X * X + Y * Y <= 128.0 ** 2).unsqueeze(0).expand(spec.vol_shape)
    out = {}
    reps = 3
    nbytes = ph.workspace_bytes_3d(g, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    for name, dt in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        v = vol.to(dt).contiguous()
        p = torch.empty((spec.n_proj,) + tuple(spec.det_shape), dtype=dt, device=dev)
        rec = torch.empty(tuple(spec.vol_shape), dtype=dt, device=dev)
        ph.fdk_cone3d(g, mats, ph.project_cone3d(g, mats, v, out=p), out=rec, ws=ws)   # warm-up
        torch.cuda.synchronize()
        fp_ms, fdk_ms = [], []
        for _ in range(reps):     # outputs and workspace preallocated: only the kernels are timed
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            ph.project_cone3d(g, mats, v, out=p)
            ev[1].record()
            ph.fdk_cone3d(g, mats, p, out=rec, ws=ws)
            ev[2].record()
            torch.cuda.synchronize()
            fp_ms.append(ev[0].elapsed_time(ev[1]))
            fdk_ms.append(ev[1].elapsed_time(ev[2]))
        d = (rec.double() - vol.double())[mask]
        out[name] = {"rmse": float(d.pow(2).mean().sqrt()), "fp_ms": sorted(fp_ms)[reps // 2],
                     "fdk_ms": sorted(fdk_ms)[reps // 2],
                     "bytes": {"volume": v.numel() * v.element_size(), "projections": p.numel() * p.element_size()}}
        del p, rec, v, d
        torch.cuda.empty_cache()
    line = {
        "metric": "FDK reconstruction RMSE and time with FP16 / BF16 storage vs FP32 (FP32 arithmetic)",
        "value": out["f16"]["rmse"] / out["f32"]["rmse"], "unit": "RMSE ratio f16/f32", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f32 arithmetic; f32/f16/bf16 storage",
        "data": "synthetic: 12 seeded random ellipsoids",
        "config": {"workload": "cone3d 512^3 at 0.5 mm, 360 views over 360 deg, 1024x768 detector at 0.8 mm",
                   "rmse_region": "inscribed cylinder r <= 128 mm, all slices"},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def adjoint_main(args):
    """The 512^3 operators as differentiable layers with the matched pairing:
    one step is a forward projection and its backward pass (A^T of the
    incoming gradient) plus a back-projection and its backward pass (B^T),
    driven through torch.autograd.  Each kernel is also timed on its own with
    HIP events over the same launches, and reported against the VALU model
    of the operator it transposes (A^T visits the forward projector's
    samples, B^T the back-projector's voxel-view updates)."""
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config(args.config)
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    prm = synth.random_ellipsoids(spec.seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
    vol = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=1, device=dev,
                                     dtype=torch.float32).contiguous()
    gen = torch.Generator(device=dev).manual_seed(5)
    w_proj = torch.randn((spec.n_proj,) + tuple(spec.det_shape), device=dev, generator=gen)   # dL/dp
    w_vol = torch.randn(tuple(spec.vol_shape), device=dev, generator=gen)                     # dL/dx
    q = ph.project_cone3d(g, mats, vol).requires_grad_(True)
    x = vol.clone().requires_grad_(True)

    def step():
        x.grad = None
        q.grad = None
        p = ph.autograd.project(x, g, mats)
        p.backward(w_proj)                 # x.grad = A^T w_proj
        r = ph.autograd.backproject(q, g, mats)
        r.backward(w_vol)                  # q.grad = B^T w_vol

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps

    # each kernel alone, into preallocated outputs
    out_p = torch.empty_like(w_proj)
    out_v = torch.empty_like(w_vol)
    calls = {"fp_cone": lambda: ph.project_cone3d(g, mats, vol, out=out_p),
             "fpT_cone": lambda: ph.project_adjoint_cone3d(g, mats, w_proj, out=out_v),
             "bp_cone": lambda: ph.backproject_cone3d(g, mats, q.detach(), out=out_v),
             "bpT_cone": lambda: ph.backproject_adjoint_cone3d(g, mats, w_vol, out=out_p)}
    ms = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
        for k in range(args.steps):
            ev[2 * k].record()
            fn()
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        ms[name] = float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)]))
    nz, ny, nx = spec.vol_shape
    updates = nx * ny * nz * spec.n_proj
    samples = count_samples(spec, dev)
    kernels = {}
    for name, units, ops, uname in (("fp_cone", samples, OPS_PER_SAMPLE, "ray samples"),
                                    ("fpT_cone", samples, OPS_PER_SAMPLE, "ray samples (transposed)"),
                                    ("bp_cone", updates, OPS_PER_UPDATE, "voxel-view updates"),
                                    ("bpT_cone", updates, OPS_PER_UPDATE, "voxel-view updates (transposed)")):
        ach = ops * units / (ms[name] * 1e-3) / 1e12
        kernels[name] = {"bound": "alu", "ms": ms[name], "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "Tops/s",
                         "frac": ach / PEAK_VALU_TOPS, "units_per_launch": units, "unit_name": uname,
                         "ops_per_unit": ops, "traffic": measured_traffic(name)}
        add_hbm(kernels[name], 4 * (nx * ny * nz + spec.n_proj * int(np.prod(spec.det_shape))))
    dom_name = max(("fpT_cone", "bpT_cone"), key=lambda n: kernels[n]["ms"])
    dom = kernels[dom_name]
    line = {
        "metric": "matched adjoint throughput at 512^3: A^T Gsamples/s and B^T GUPS (autograd backward)",
        "value": samples / (ms["fpT_cone"] * 1e-3) / 1e9, "unit": "Gsamples/s (A^T)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: 12 seeded random ellipsoids and seeded Gaussian gradients, resident in HBM",
        "config": {"workload": f"cone3d {nx}x{ny}x{nz} at {spec.vol_spacing[0]} mm, {spec.n_proj} views, "
                               f"{spec.det_shape[1]}x{spec.det_shape[0]} detector at {spec.det_spacing[0]} mm",
                   "step": "autograd: A forward + A^T backward, B forward + B^T backward"},
        "fpT_gsamples_per_s": samples / (ms["fpT_cone"] * 1e-3) / 1e9,
        "bpT_gups": updates / (ms["bpT_cone"] * 1e-3) / 1e9,
        "fpT_over_fp": ms["fpT_cone"] / ms["fp_cone"], "bpT_over_bp": ms["bpT_cone"] / ms["bp_cone"],
        "roofline": {"kernel": dom_name, "bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                     "unit": dom["unit"], "frac": dom["frac"], "traffic": dom["traffic"]},
        "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): each GPU would run this same path "
              "on its own share of the views (projections) or z-slabs (volume).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "adjoint":
        adjoint_main(args)
        return
    if args.workload == "corrector":
        corrector_main(args)
        return
    if args.workload == "tv":
        tv_main(args)
        return
    if args.workload == "filter2d":
        filter2d_main(args)
        return
    if args.workload == "precision":
        precision_main(args)
        return
    if args.workload == "fan2d":
        fan2d_main(args)
        return
    if args.workload == "copyref":
        import torch
        x = torch.ones(COPY_BYTES // 4, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copyref", "bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES}), flush=True)
        return
    import numpy as np
    import torch

    import paper_1904_13342_amd as ph
    import synth

    dev = torch.device("cuda:0")
    spec = synth.config(args.config)
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    prm = synth.random_ellipsoids(spec.seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
    vol = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=1, device=dev,
                                     dtype=torch.float32).contiguous()
    proj = torch.empty((spec.n_proj,) + tuple(spec.det_shape), dtype=torch.float32, device=dev)
    q = torch.empty_like(proj)
    rec = torch.empty_like(vol)
    torch.cuda.synchronize()

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        ph.project_cone3d(g, mats, vol, out=proj)
        if ev is not None:
            ev[1].record()
        ph.weight_filter_3d(g, proj, out=q)
        if ev is not None:
            ev[2].record()
        ph.backproject_cone3d(g, mats, q, out=rec)
        if ev is not None:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fp_ms = np.mean([e[0].elapsed_time(e[1]) for e in events])
    wf_ms = np.mean([e[1].elapsed_time(e[2]) for e in events])
    bp_ms = np.mean([e[2].elapsed_time(e[3]) for e in events])
    ms_per_step = wall * 1e3 / args.steps

    nz, ny, nx = spec.vol_shape
    nv, nu = spec.det_shape
    updates = nx * ny * nz * spec.n_proj
    samples = count_samples(spec, dev)
    fdk_ms = wf_ms + bp_ms
    bp_gups = updates / (bp_ms * 1e-3) / 1e9
    fdk_gups = updates / (fdk_ms * 1e-3) / 1e9
    fp_gsps = samples / (fp_ms * 1e-3) / 1e9
    wf_bytes = 2 * 4 * spec.n_proj * nv * nu + 4 * spec.n_proj * nu

    kernels = {
        "fp_cone": {"bound": "alu", "ms": fp_ms, "achieved": OPS_PER_SAMPLE * samples / (fp_ms * 1e-3) / 1e12,
                    "peak": PEAK_VALU_TOPS, "unit": "Tops/s", "units_per_launch": samples,
                    "unit_name": "ray samples", "ops_per_unit": OPS_PER_SAMPLE},
        "weight_filter": {"bound": "hbm", "ms": wf_ms, "achieved": wf_bytes / (wf_ms * 1e-3) / 1e9,
                          "peak": PEAK_HBM_GBS, "unit": "GB/s", "units_per_launch": wf_bytes,
                          "unit_name": "bytes"},
        "bp_cone": {"bound": "alu", "ms": bp_ms, "achieved": OPS_PER_UPDATE * updates / (bp_ms * 1e-3) / 1e12,
                    "peak": PEAK_VALU_TOPS, "unit": "Tops/s", "units_per_launch": updates,
                    "unit_name": "voxel-view updates", "ops_per_unit": OPS_PER_UPDATE},
    }
    vol_bytes, proj_bytes = 4 * nx * ny * nz, 4 * spec.n_proj * nv * nu
    for name, kv in kernels.items():
        kv["frac"] = kv["achieved"] / kv["peak"]
        kv["traffic"] = measured_traffic(name)
    # the projector and back-projector are VALU-bound; their HBM figures are diagnostics
    add_hbm(kernels["fp_cone"], vol_bytes + proj_bytes)
    add_hbm(kernels["bp_cone"], vol_bytes + proj_bytes)
    dom_name = max(kernels, key=lambda n: kernels[n]["ms"])
    dom = kernels[dom_name]
    roofline = {"kernel": dom_name, "bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                "unit": dom["unit"], "frac": dom["frac"], "traffic": dom["traffic"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, vol.cpu().numpy(), args.cpu_seconds)

    line = {
        "metric": "cone-beam backprojection GUPS + forward-proj Gsamples/s at 512^3; %HBM roofline",
        "value": fdk_gups,
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: 12 seeded random ellipsoids, resident in HBM",
        "config": {"workload": f"{spec.kind} {nx}x{ny}x{nz} at {spec.vol_spacing[0]} mm, {spec.n_proj} views over "
                               f"{round(math.degrees(spec.angular_range))} deg, {nu}x{nv} detector at "
                               f"{spec.det_spacing[0]} mm, SID {spec.sid:g}, SDD {spec.sdd:g}",
                   "batch": 1, "step": "forward projection + weighting/Ram-Lak filter + back-projection"},
        "bp_gups": bp_gups,
        "fdk_gups": fdk_gups,
        "fp_gsamples_per_s": fp_gsps,
        "fp_ms": fp_ms,
        "weight_filter_ms": wf_ms,
        "bp_ms": bp_ms,
        "fp_samples": samples,
        "bp_updates": updates,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
