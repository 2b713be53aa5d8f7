"""Benchmark: Myrtle-10 NNGP Gram block (32x32x3 images, 4096 x 4096) on one
MI355X through libnk.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one nk_myrtle_nngp call on the whole block (variance tables, the
three fused stage kernels, readout and block write) with the images already
in device memory.  Beside it the run times one forward + backward pass of the
differentiable workload (Myrtle-5 at 32x32x3: kernel ridge regression of 256
learnable support images onto 2048 target images, gradients with respect to
the support pixels and both sigmas) and reports it as fwd+bwd pairs/s.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

T0 = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Myrtle-10 NNGP kernel entries/s at 32x32x3; fwd+bwd pairs/s; %FP32 VALU peak"
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 CU x 2.4 GHz x 256 flop/clk (packed FMA, 64 lanes)
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense fp32 matrix-core peak of MI355X
PMC_FILE = os.path.join(ROOT, "profiles", "myrtle_stage1_n32_hbm_counters.md")
PCG_PMC_FILE = os.path.join(ROOT, "profiles", "pcg_kmv_32768_hbm_counters.md")
PCG_SRC = os.path.join(ROOT, "paper_2303_05420_amd", "csrc", "pcg.hip")
# the sources the stage-1 kernel is compiled from (its counters are void once any of them changes)
STAGE_SRCS = [os.path.join(ROOT, "paper_2303_05420_amd", "csrc", f)
              for f in ("stage32.hip", "stage_kernel.h", "nk_tile.h", "nk_common.h")]
VALU_PMC_FILE = os.path.join(ROOT, "profiles", "myrtle_stage1_n32_valu_counters.md")


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=4096, help="block side (the headline workload is 4096)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=48, help="side of the oracle sample sub-block")
    p.add_argument("--copy-calib-mib", type=int, default=0,
                   help="also run a plain device copy of this many MiB (counter calibration runs)")
    p.add_argument("--no-fwd-bwd", action="store_true", help="skip the fwd+bwd measurement")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain tile comparison")
    p.add_argument("--no-ntk", action="store_true", help="skip the Myrtle-10 NTK measurement")
    p.add_argument("--no-pcg", action="store_true", help="skip the preconditioned-CG solve measurement")
    p.add_argument("--no-cv8", action="store_true", help="skip the CV8 NNGP measurement")
    p.add_argument("--no-approx", action="store_true", help="skip the approximate-solver measurement")
    p.add_argument("--no-64", action="store_true", help="skip the 64x64 Myrtle-7 block")
    p.add_argument("--budget-s", type=float, default=450.0,
                   help="wall-clock budget of the whole run from process start (s); timed headline steps stop "
                        "after at least three once --headline-share of it is used, side legs that would end "
                        "past it are skipped by name")
    p.add_argument("--headline-share", type=float, default=0.55)
    p.add_argument("--batched-reps", type=int, default=3, help="timed passes of each form (median reported)")
    p.add_argument("--batched-full", action="store_true",
                   help="batched comparison at full size (64 tiles, sides 32..2048, about 7e7 pairs; minutes)")
    return p.parse_args()


def _src_hash(path) -> str:
    h = hashlib.sha256()
    for q in ([path] if isinstance(path, str) else path):
        h.update(open(q, "rb").read())
    return h.hexdigest()[:16]


def _summary_json(path: str):
    """The machine-readable block of a committed counter summary, or None."""
    try:
        text = open(path).read()
        return json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None


def _traffic(stage_launch_pairs: int):
    """HBM bytes per stage-1 launch from the committed counter summary, or None
    when there is none or the kernel source changed since it was taken."""
    d = _summary_json(PMC_FILE)
    if d is None or d.get("stage_src_sha256_16") != _src_hash(STAGE_SRCS):
        return None
    per_pair = d.get("hbm_bytes_per_pair")
    if per_pair is None:
        return None
    return float(per_pair) * stage_launch_pairs


def _valu_counters():
    """VALU counters of the stage-1 kernel from the committed summary (issued
    FP32 flops against the op model, VALU busy), or None when there is none
    or the kernel's sources changed since they were taken."""
    d = _summary_json(VALU_PMC_FILE)
    if d is None or d.get("stage_src_sha256_16") != _src_hash(STAGE_SRCS):
        return None
    return {k: d[k] for k in ("valu_busy_pct", "issued_over_algorithmic_flops", "valu_instructions_per_entry_layer",
                              "fp32_instruction_mix") if k in d}


def _pcg_traffic(n: int):
    """HBM bytes per K.P launch from the committed counter summary, or None when
    there is none, it was taken at another size, or pcg.hip changed since."""
    try:
        text = open(PCG_PMC_FILE).read()
        d = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    if d.get("pcg_src_sha256_16") != _src_hash(PCG_SRC) or d.get("n") != n:
        return None
    return d.get("hbm_bytes_per_dispatch")


def _fwd_bwd(torch):
    """One timed forward + backward pass of the kernel-ridge-regression loss
    through the Myrtle-5 NNGP (after one untimed pass); the ALU roofline of
    the first stage's adjoint kernel under the adjoint op model."""
    import synth
    from paper_2303_05420_amd import _lib, krr_grad, workmodel

    w = synth.WORKLOADS["myrtle5_krr_grad"]
    ns, nt = w["n_support"], w["n_target"]
    xs = torch.from_numpy(synth.correlated_images(ns, 32, 32, 3, w["length"], w["seeds"][0])).cuda()
    xt = torch.from_numpy(synth.correlated_images(nt, 32, 32, 3, w["length"], w["seeds"][1])).cuda()
    ys = torch.from_numpy(synth.balanced_labels(ns, 10)).cuda()
    yt = torch.from_numpy(synth.teacher_labels(synth.correlated_images(nt, 32, 32, 3, w["length"], w["seeds"][1]),
                                               10, w["seeds"][2])).cuda()

    # Keep the first-stage outputs of every pair between the forward and the
    # adjoint pass (146 GB at this size) when the device has room for them.
    cfg = _lib.myrtle_cfg(32, 3, w["depth"], w["sigma_w2"], w["sigma_b2"])
    keep_bytes = int(_lib.lib().nk_krr_mse_grad_workspace_keep(ctypes.byref(cfg), ns, nt, 10))
    keep = torch.cuda.mem_get_info()[0] > keep_bytes + (8 << 30)

    def run():
        return krr_grad.krr_mse_loss_and_grad(xs, ys, xt, yt, w["depth"], w["sigma_w2"], w["sigma_b2"],
                                              w["ridge_rel"], keep_checkpoints=keep)

    try:
        run()
    except torch.cuda.OutOfMemoryError:
        from paper_2303_05420_amd import ops
        keep = False
        ops.release_workspace()
        torch.cuda.empty_cache()
        run()
    torch.cuda.synchronize()
    print(f"fwd+bwd warm-up done (first-stage outputs kept: {keep})", file=sys.stderr, flush=True)
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    loss, dxs, ds, lam = run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    pairs = ns * (ns + 1) // 2 + nt * ns
    fwd_ms = sum(v[1] for k, v in prof.items() if k.startswith("myrtle_stage") and not k.endswith("_bwd"))
    bwd_ms = sum(v[1] for k, v in prof.items() if k.endswith("_bwd"))
    print(f"fwd+bwd: {dt * 1e3:.1f} ms for {pairs} pairs", file=sys.stderr, flush=True)
    launches, kms = prof["myrtle_stage1_n32_bwd"]
    flop_pair = workmodel.adjoint_first_stage_flops_per_pair(32, 3, w["depth"][0])
    achieved = flop_pair * pairs / (kms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None, "kernel": "myrtle_stage1_n32_bwd",
            "avg_launch_ms": round(kms / launches, 3), "launches": launches, "flops_per_pair": flop_pair}
    return {"value": round(pairs / dt, 3), "unit": "pairs/s", "pairs": pairs, "ms": round(dt * 1e3, 3),
            "workload": f"Myrtle-5 NNGP at 32x32x3, KRR of {ns} learnable support images onto {nt} targets "
                        f"(K_ss symmetric + K_ts), loss + d/d(support pixels) + d/d(sigma_w2, sigma_b2)",
            "loss": loss, "dsigma": [float(v) for v in ds.cpu().tolist()],
            "first_stage_outputs": (f"kept between the passes ({keep_bytes / 1e9:.1f} GB workspace)" if keep
                                    else "recomputed in the adjoint pass"),
            "kernels_ms": {k: round(v[1], 3) for k, v in prof.items()},
            "stage_kernels_fwd_ms": round(fwd_ms, 3), "stage_kernels_bwd_ms": round(bwd_ms, 3), "roofline": roof}


def _ntk(torch, n: int = 1024):
    """Myrtle-10 neural tangent kernel (with its NNGP) on an n x n block of the
    headline images, timed once after an untimed 64 x 64 pass; the first-stage
    kernel's ALU roofline under the tangent-kernel op model."""
    import synth
    from paper_2303_05420_amd import _lib, ops, workmodel

    w = synth.WORKLOADS["myrtle10_32x32_4096"]
    x1 = torch.from_numpy(synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][0])).cuda()
    x2 = torch.from_numpy(synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][1])).cuda()
    ops.myrtle_ntk(x1[:64], x2[:64], w["depth"], w["sigma_w2"], w["sigma_b2"])
    torch.cuda.synchronize()
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    ops.myrtle_ntk(x1, x2, w["depth"], w["sigma_w2"], w["sigma_b2"], with_nngp=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    print(f"ntk: {dt:.2f} s for {n * n} pairs", file=sys.stderr, flush=True)
    launches, kms = prof["myrtle_ntk_stage1_n32"]
    flop_pair = workmodel.ntk_first_stage_flops_per_pair(32, 3, w["depth"][0])
    achieved = flop_pair * n * n / (kms / 1e3) / 1e12
    return {"value": round(n * n / dt, 3), "unit": "pairs/s", "pairs": n * n, "ms": round(dt * 1e3, 3),
            "workload": f"Myrtle-10 NTK and NNGP together, 32x32x3, one {n}x{n} block of the headline images",
            "kernels_ms": {k: round(v[1], 3) for k, v in prof.items()},
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                         "kernel": "myrtle_ntk_stage1_n32", "avg_launch_ms": round(kms / launches, 3),
                         "pairs_per_launch": n * n // launches, "flops_per_pair": flop_pair}}


def _myrtle64(torch):
    """The 256 x 256 Myrtle-7 block on 64x64x3 images (length scale 6 px) of the
    uneven-tile workload: one untimed and one timed call; the 64x64 first-stage
    kernel's ALU roofline under the op model."""
    import synth
    from paper_2303_05420_amd import _lib, ops, workmodel

    w = synth.WORKLOADS["myrtle7_uneven64"]
    n, hw, depth = w["big_n"], w["big_hw"], w["depth"]
    x1 = torch.from_numpy(synth.correlated_images(n, hw, hw, 3, w["big_length"], w["big_seeds"][0])).cuda()
    x2 = torch.from_numpy(synth.correlated_images(n, hw, hw, 3, w["big_length"], w["big_seeds"][1])).cuda()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ops.myrtle_nngp(x1, x2, depth, w["sigma_w2"], w["sigma_b2"], out=out)
    torch.cuda.synchronize()
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    ops.myrtle_nngp(x1, x2, depth, w["sigma_w2"], w["sigma_b2"], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    launches, kms = prof[f"myrtle_stage1_n{hw}"]
    flop_pair = (workmodel.FLOPS_PER_ENTRY_LAYER * depth[0] * hw ** 4
                 + workmodel.FLOPS_PER_SEED_ENTRY_PER_CHANNEL * 3 * hw ** 4
                 + workmodel.FLOPS_PER_POOLED_ENTRY * hw ** 4)
    achieved = flop_pair * n * n / (kms / 1e3) / 1e12
    print(f"myrtle7 64x64: {dt * 1e3:.1f} ms for {n * n} pairs", file=sys.stderr, flush=True)
    return {"workload": f"Myrtle-7 NNGP, 64x64x3 correlated images (length scale 6 px), one {n}x{n} block",
            "value": round(n * n / dt, 1), "unit": "entries/s", "ms": round(dt * 1e3, 3),
            "kernels_ms": {k: round(v[1], 3) for k, v in prof.items()},
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                         "kernel": f"myrtle_stage1_n{hw}", "avg_launch_ms": round(kms / launches, 3),
                         "pairs_per_launch": n * n // launches}}


def _batched(torch, full: bool, reps: int = 3):
    """Uneven Myrtle-7 tiles at 32x32x3: the batched pass (tuned schedule,
    hipGraph) against the plain form (one nk_myrtle_nngp call per tile).
    One untimed pass of each, then `reps` timed passes of each, alternating;
    medians and ranges are reported and the outputs compared bitwise."""
    import synth
    from paper_2303_05420_amd import ops

    w = synth.WORKLOADS["myrtle7_uneven64"]
    depth = w["depth"]
    hi = w["hi"] if full else 512
    pool = w["pool"] if full else 512
    shapes = synth.uneven_tile_shapes(w["n_tiles"], w["lo"], hi, w["seeds"][2])
    xa = torch.from_numpy(synth.correlated_images(pool, 32, 32, 3, w["length"], w["seeds"][0])).cuda()
    xb = torch.from_numpy(synth.correlated_images(pool, 32, 32, 3, w["length"], w["seeds"][1])).cuda()
    outs_b = [torch.empty((int(a), int(b)), dtype=torch.float32, device="cuda") for a, b in shapes]
    outs_p = [torch.empty_like(o) for o in outs_b]
    tiles = [(xa[:int(a)], xb[:int(b)], o) for (a, b), o in zip(shapes, outs_b)]
    pairs = int(sum(int(a) * int(b) for a, b in shapes))

    def plain():
        for (a, b), o in zip(shapes, outs_p):
            ops.myrtle_nngp(xa[:int(a)], xb[:int(b)], depth, out=o)

    def batched():
        ops.myrtle_nngp_batched(tiles, depth, graph=True)

    fns = {"batched": batched, "plain": plain}
    for name, fn in fns.items():
        fn()
        torch.cuda.synchronize()
        print(f"{name} tiles: warm-up done", file=sys.stderr, flush=True)
    times = {"batched": [], "plain": []}
    for r in range(max(1, reps)):
        for name, fn in fns.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times[name].append(time.perf_counter() - t0)
            print(f"{name} tiles pass {r + 1}: {times[name][-1]:.3f} s", file=sys.stderr, flush=True)
    same = all(torch.equal(a, b) for a, b in zip(outs_b, outs_p))
    cands, chosen = ops.batched_tuning(32, 3, depth)

    def med(v):
        s = sorted(v)
        k = len(s)
        return s[k // 2] if k % 2 else 0.5 * (s[k // 2 - 1] + s[k // 2])

    mb, mp = med(times["batched"]), med(times["plain"])
    return {"workload": f"Myrtle-7 NNGP at 32x32x3, {len(shapes)} tiles with sides U{{{w['lo']}..{hi}}} "
                        f"over prefixes of two pools of {pool} images",
            "pairs": pairs, "passes_each": len(times["batched"]),
            "batched_pairs_per_s": round(pairs / mb, 1), "plain_pairs_per_s": round(pairs / mp, 1),
            "batched_s": [round(v, 4) for v in times["batched"]], "plain_s": [round(v, 4) for v in times["plain"]],
            "speedup_median": round(mp / mb, 4),
            "ranges_disjoint": bool(max(times["batched"]) < min(times["plain"])
                                    or max(times["plain"]) < min(times["batched"])),
            "bitwise_equal": bool(same), "schedule": chosen, "candidates_tried": len(cands),
            "shape_candidates_us_per_pair": {f"x{c['wg_pairs_mult']}": round(c["us_per_pair"], 4)
                                             for c in cands if c["kind"] == "shape"}}


def _cv8(torch, cpu: bool):
    """CV8 NNGP (CNN-VEC, depth 8, flatten readout) on one 4096 x 4096 block of
    32x32x3 images: one untimed and one timed call, the pair kernel's ALU
    roofline, and the FP64 oracle on a 64 x 64 sub-block with its parity."""
    import numpy as np

    import synth
    from paper_2303_05420_amd import _lib, ops, workmodel

    w = synth.WORKLOADS["cv8_32x32_4096"]
    n, hw, depth = w["n1"], w["hw"], w["depth"]
    xa = synth.correlated_images(n, hw, hw, 3, w["length"], w["seeds"][0])
    xb = synth.correlated_images(n, hw, hw, 3, w["length"], w["seeds"][1])
    ta, tb = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ops.cv_nngp(ta, tb, depth, w["sigma_w2"], w["sigma_b2"], out=out)
    torch.cuda.synchronize()
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    ops.cv_nngp(ta, tb, depth, w["sigma_w2"], w["sigma_b2"], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    kern = f"cv_pairs_n{hw}"
    launches, kms = prof[kern]
    flops = workmodel.cv_flops_per_pair(hw, 3, depth) * n * n
    achieved = flops / (kms / launches / 1e3) / 1e12
    res = {"workload": f"CV8 NNGP (CNN-VEC depth 8, flatten readout), 32x32x3 correlated images, one {n}x{n} block",
           "value": round(n * n / dt, 1), "unit": "entries/s", "ms": round(dt * 1e3, 3),
           "kernels_ms": {k: round(v[1], 3) for k, v in prof.items()},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": kern, "avg_launch_ms": round(kms / launches, 3)}}
    print(f"cv8: {dt * 1e3:.1f} ms for {n * n} entries", file=sys.stderr, flush=True)
    if cpu:
        import oracle

        m = 64
        t0 = time.perf_counter()
        q1, d1 = oracle.cv_self(xa[:m], depth, w["sigma_w2"], w["sigma_b2"])
        q2, d2 = oracle.cv_self(xb[:m], depth, w["sigma_w2"], w["sigma_b2"])
        a, b = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        ref = oracle.cv_pairs(xa[:m], xb[:m], np.stack([a.ravel(), b.ravel()], 1), depth, w["sigma_w2"],
                              w["sigma_b2"], q1, q2).reshape(m, m)
        cdt = time.perf_counter() - t0
        err = float(np.max(np.abs(out[:m, :m].cpu().numpy() - ref) / np.sqrt(np.outer(d1, d2))))
        res["cpu_baseline"] = {"value": round(m * m / cdt, 1), "unit": "entries/s", "kind": "oracle",
                               "cores": _host_threads(),
                               "sample": f"{m}x{m} sub-block of the same block plus its {2 * m} self recursions"}
        res["parity"] = {"max_normalised_error": err, "entries": m * m, "tolerance": 2e-5}
    return res


def _approx(torch):
    """The four approximate solvers on 32768 training points (FC-3 NNGP of the
    PCG workload's images) and 2048 test images: Nystrom and SoR with a random
    subset of 2048, block-diagonal and the committee machine with a random
    partition into 16 blocks of 2048.  Kernel blocks are built on the GPU
    before the timed calls; each method is timed once after an untimed call.
    Model flops (multiply-adds counted twice) of each method's float64
    products and factorisations are reported against the 78.6 TFLOP/s FP64
    vector peak."""
    import numpy as np

    import synth
    from paper_2303_05420_amd import ops

    w = synth.WORKLOADS["fc3_approx_32768"]
    n, m, r, p = w["n"], w["m"], w["rank"], w["blocks"]
    c = w["n_classes"]
    xs = synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][0])
    xt = synth.correlated_images(m, 32, 32, 3, w["length"], w["seeds"][3])
    y = torch.from_numpy(synth.teacher_labels(xs, c, w["seeds"][1])).cuda()
    x = torch.from_numpy(xs.reshape(n, -1)).cuda()
    xm = torch.from_numpy(xt.reshape(m, -1)).cuda()
    fc = dict(depth=w["fc_depth"], sigma_w2=w["fc_sigma_w2"], sigma_b2=w["fc_sigma_b2"])
    rng = np.random.default_rng(w["seeds"][2])
    sub = torch.from_numpy(rng.choice(n, r, replace=False)).cuda()
    perm = torch.from_numpy(np.random.default_rng(w["seeds"][4]).permutation(n)).cuda()
    k_nr = ops.fc_nngp(x, x[sub].contiguous(), **fc)
    k_rr = ops.fc_nngp(x[sub].contiguous(), None, **fc)
    k_mn = ops.fc_nngp(xm, x, **fc)
    k_mr = k_mn[:, sub].contiguous()
    k_mm = ops.fc_nngp(xm, None, **fc)
    diag_mean = float(torch.diagonal(k_rr).double().mean())  # lambda from the subset's diagonal
    lam = w["ridge_rel"] * diag_mean
    xp = x[perm].contiguous()
    yp = y[perm].contiguous()
    b = n // p
    blocks = [ops.fc_nngp(xp[i * b:(i + 1) * b].contiguous(), None, **fc) for i in range(p)]
    k_mp = k_mn[:, perm].contiguous()
    runs = {
        "nystrom": (lambda: ops.krr_nystrom(k_nr, k_rr, k_mn, y, lam, w["jitter"]),
                    2.0 * n * r * r + 2.0 * n * r * c * 2 + r ** 3 / 3 + 2.0 * m * n * c),
        "sor": (lambda: ops.krr_sor(k_nr, k_rr, k_mr, y, lam, w["jitter"]),
                2.0 * n * r * r + 2.0 * n * r * c + r ** 3 / 3 + 2.0 * m * r * c),
        "block_diag": (lambda: ops.krr_block_diag(blocks, k_mp, yp, lam),
                       p * (b ** 3 / 3 + 2.0 * b * b * c) + 2.0 * m * n * c),
        "bcm": (lambda: ops.krr_bcm(blocks, k_mp, k_mm, yp, lam, w["jitter"]),
                p * (b ** 3 / 3 + 2.0 * b * b * (c + m) + 2.0 * m * b * (c + m) + m ** 3 / 3 + 2.0 * m ** 3)
                + 4.0 * m ** 3 / 3),
    }
    out = {"workload": f"approximate KRR on {n} training points (FC-3 NNGP of 32x32x3 correlated images), "
                       f"{m} test points, {c} targets: Nystrom / SoR with a random subset of {r}, block-diagonal / "
                       f"committee machine with a random partition into {p} blocks of {b}",
           "lambda": lam}
    for name, (fn, flops) in runs.items():
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"ms": round(dt * 1e3, 3), "model_tflops": round(flops / dt / 1e12, 3),
                     "frac_fp64_peak": round(flops / dt / 1e12 / 78.6, 4)}
        print(f"approx {name}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return out


def _pcg(torch, cpu: bool):
    """Kernel regression by FP64 preconditioned CG on a 32768 x 32768 float32
    Gram (FC-3 NNGP of the workload's images, built on the GPU before the
    timed region), 10 targets, rank-512 pivoted-Cholesky preconditioner,
    tol 1e-8: one untimed solve, one timed solve, then 20 profiled K.P
    products for the HBM roofline.  With cpu, the FP64 oracle solves the
    leading 4096 x 4096 sub-system of the same K on the host, beside the GPU
    solve of that sub-system."""
    import numpy as np

    import synth
    from paper_2303_05420_amd import _lib, ops

    w = synth.WORKLOADS["fc3_pcg_32768"]
    n = w["n"]
    xs = synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][0])
    y = torch.from_numpy(synth.teacher_labels(xs, w["n_classes"], w["seeds"][1]).astype(np.float64)).cuda()
    xg = torch.from_numpy(xs.reshape(n, -1)).cuda()
    ops.fc_nngp(xg[:256], None, w["fc_depth"], w["fc_sigma_w2"], w["fc_sigma_b2"])  # untimed first call
    torch.cuda.synchronize()
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    k = ops.fc_nngp(xg, None, w["fc_depth"], w["fc_sigma_w2"], w["fc_sigma_b2"])
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    fc_launches, fc_ms = _lib.profile_read(reset=True)["fc_nngp"]
    d_in = int(xg.shape[1])
    del xg
    # the block is symmetric: its distinct entries are n (n + 1) / 2, and the
    # kernel runs the tiles on and above the diagonal and mirrors them
    fc_flops = 2.0 * d_in * n * (n + 1) / 2
    fc_tflops = fc_flops / (fc_ms / 1e3) / 1e12
    fc_gram = {"workload": f"FC-3 NNGP Gram of {n} 32x32x3 correlated images (d = {d_in}), {n}x{n}, "
                           f"sigma_w2={w['fc_sigma_w2']}, sigma_b2={w['fc_sigma_b2']}",
               "value": round(n * n / (fc_ms / 1e3), 1), "unit": "entries/s", "ms": round(fc_ms, 3),
               "roofline": {"bound": "mfma", "achieved": round(fc_tflops, 3), "peak": FP32_MFMA_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": round(fc_tflops / FP32_MFMA_PEAK_TFLOPS, 4),
                            "traffic": None, "kernel": "fc_kernel (first-layer contraction on fp32 MFMA, ReLU "
                                                       "recursion in its epilogue; the two diagonal kernels "
                                                       "are inside the timed scope)",
                            "avg_launch_ms": round(fc_ms / fc_launches, 3),
                            "flops_per_launch": fc_flops}}
    print(f"fc3 gram: {fc_ms:.1f} ms for {n}x{n}", file=sys.stderr, flush=True)
    kt = k.t().contiguous()
    k.add_(kt).mul_(0.5)  # exactly symmetric (the solver reads rows as columns)
    del kt

    def solve(kk, yy):
        return ops.krr_pcg(kk, yy, w["ridge_rel"], True, rank=w["rank"], tol=w["tol"], max_iter=w["max_iter"])

    solve(k, y)
    torch.cuda.synchronize()
    print("pcg warm-up done", file=sys.stderr, flush=True)
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    t0 = time.perf_counter()
    x, iters, relres, st = solve(k, y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    print(f"pcg: {dt * 1e3:.1f} ms, {int(iters.max())} iterations", file=sys.stderr, flush=True)

    p = torch.randn(n, w["n_classes"], dtype=torch.float64, device="cuda")
    ops.gram_matvec(k, p, st["lambda"])
    torch.cuda.synchronize()
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    for _ in range(20):
        ops.gram_matvec(k, p, st["lambda"])
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    mv = _lib.profile_read(reset=True)["gram_matvec"]
    mv_ms = mv[1] / mv[0]
    bytes_per_launch = 4.0 * n * n  # each float32 entry of K read once
    achieved = bytes_per_launch / (mv_ms / 1e3) / 1e9
    setup_ms = sum(prof.get(kk, (0, 0.0))[1] for kk in ("pivoted_cholesky", "pcg_precond_setup"))
    it_max = int(iters.max())
    out = {"workload": f"kernel ridge regression, FP64 preconditioned CG on a {n}x{n} float32 Gram "
                       f"(FC-3 NNGP of 32x32x3 correlated images), {w['n_classes']} one-hot targets, "
                       f"ridge {w['ridge_rel']} mean diag, pivoted-Cholesky rank {w['rank']}, tol {w['tol']}",
           "n": n, "targets": w["n_classes"], "rank": st["rank"], "tol": w["tol"], "iterations": it_max,
           "max_relres": float(relres.max()), "solve_ms": round(dt * 1e3, 3),
           "setup_ms": round(setup_ms, 3), "ms_per_iteration": round((dt * 1e3 - setup_ms) / max(it_max, 1), 4),
           "kernels_ms": {kk: round(v[1], 3) for kk, v in prof.items()},
           "fc_gram": fc_gram,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(achieved / 8000.0, 4), "traffic": _pcg_traffic(n),
                        "kernel": f"kmv_partial_kernel<{w['n_classes']}, true> (K.P)",
                        "avg_launch_ms": round(mv_ms, 4), "algorithmic_bytes_per_launch": bytes_per_launch}}
    if cpu:
        from oracle import solvers

        m = w["cpu_n"]
        ks = k[:m, :m].contiguous()
        ys = y[:m].contiguous()
        solve(ks, ys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xg, ig, _, sg = solve(ks, ys)
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        k64 = ks.cpu().numpy().astype(np.float64)
        y64 = ys.cpu().numpy()
        t0 = time.perf_counter()
        ref = solvers.pcg(k64, y64, solvers.ridge_lambda(k64, w["ridge_rel"], True), w["rank"], w["tol"],
                          w["max_iter"])
        cdt = time.perf_counter() - t0
        err = float(np.max(np.abs(xg.cpu().numpy() - ref["X"])) / np.max(np.abs(ref["X"])))
        out["cpu_baseline"] = {"value": round(cdt * 1e3, 1), "unit": "ms per solve", "kind": "oracle",
                               "cores": _host_threads(),
                               "sample": f"leading {m}x{m} sub-system of the same K and targets, same settings "
                                         f"({int(ref['iters'].max())} iterations, numpy float64)",
                               "gpu_ms_same_sample": round(gdt * 1e3, 3),
                               "gpu_iterations_same_sample": int(ig.max()),
                               "max_rel_diff_x_vs_oracle": err}
        print(f"pcg sample {m}: gpu {gdt * 1e3:.1f} ms, oracle {cdt * 1e3:.0f} ms", file=sys.stderr, flush=True)
    del k
    return out


def _host_threads() -> int:
    """Oracle threads: every core this process may run on, capped by the
    OpenMP thread count the host sets for it (the CPU share of one GPU)."""
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        cores = min(cores, int(omp))
    return max(1, cores)


def _elapsed() -> float:
    return time.perf_counter() - T0


_EMITTED = [False]


def _emit(rec: dict):
    if not _EMITTED[0]:
        _EMITTED[0] = True
        print(json.dumps(rec), flush=True)


def _on_term(rec: dict):
    def handler(signum, frame):
        rec["terminated"] = f"signal {signum} after {_elapsed():.1f} s; legs not reached are missing"
        _emit(rec)
        os._exit(128 + signum)
    return handler


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {a.gpus}); on several GPUs each would "
              "compute its own Gram blocks with no communication, so the figure would be the one-GPU rate "
              "times the GPU count.", file=sys.stderr)
        sys.exit(2)

    import signal

    import numpy as np
    import torch

    import synth
    from paper_2303_05420_amd import _lib, ops, workmodel

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    print(f"[{_elapsed():.1f} s] torch and libnk imported", file=sys.stderr, flush=True)

    w = synth.WORKLOADS["myrtle10_32x32_4096"]
    n = a.n
    depth = w["depth"]
    hw = 32
    pairs = n * n
    rec = {
        "metric": METRIC, "value": None, "unit": "entries/s", "n_gpus": 1, "steps": 0, "warmup": 0,
        "steps_requested": a.steps, "warmup_requested": a.warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Myrtle-10 NNGP, 32x32x3 correlated-Gaussian images (length scale 3 px), "
                               f"one {n}x{n} Gram block (x1 != x2), sigma_w2=2, sigma_b2=0",
                   "n1": n, "n2": n, "depth": list(depth), "pairs": pairs},
        "budget_s": a.budget_s,
        "context": "paper: ~300 GPU-hours for the full CIFAR-10 Myrtle kernel (hardware and precision not stated)",
    }
    signal.signal(signal.SIGTERM, _on_term(rec))

    x1n = synth.correlated_images(n, hw, hw, 3, w["length"], w["seeds"][0])
    x2n = synth.correlated_images(n, hw, hw, 3, w["length"], w["seeds"][1])
    x1 = torch.from_numpy(x1n).cuda()
    x2 = torch.from_numpy(x2n).cuda()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    cfg = _lib.myrtle_cfg(hw, 3, depth, w["sigma_w2"], w["sigma_b2"])
    ws = ops.workspace(ops.workspace_size(_lib.NK_OP_MYRTLE, cfg, n, n), x1.device)

    def step():
        ops.myrtle_nngp(x1, x2, depth, w["sigma_w2"], w["sigma_b2"], out=out, ws=ws)

    # Warm-up: at most one full step (the kernels are compiled ahead of time;
    # the first call only sets LDS attributes).
    warm = min(a.warmup, 1)
    for i in range(warm):
        step()
        torch.cuda.synchronize()
        print(f"[{_elapsed():.1f} s] warm-up step {i + 1}/{warm} done", file=sys.stderr, flush=True)

    # Timed steps: up to --steps, stopped early (after at least min(3, steps))
    # once the next step would end past the headline's share of the budget.
    head_deadline = a.budget_s * a.headline_share
    _lib.profile_read(reset=True)
    _lib.profile_enable(True)
    evs = [torch.cuda.Event(enable_timing=True)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    done = 0
    while done < a.steps:
        step()
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        evs.append(e)
        e.synchronize()
        done += 1
        last_s = evs[-2].elapsed_time(evs[-1]) / 1e3
        print(f"[{_elapsed():.1f} s] timed step {done}: {last_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
        if done >= min(3, a.steps) and _elapsed() + last_s > head_deadline:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _lib.profile_enable(False)
    prof = _lib.profile_read(reset=True)
    ms_each = [evs[i].elapsed_time(evs[i + 1]) for i in range(done)]
    ms_step = sum(ms_each) / done
    srt = sorted(ms_each)
    med = srt[done // 2] if done % 2 else 0.5 * (srt[done // 2 - 1] + srt[done // 2])
    print(f"timed {done} step(s): {ms_step:.1f} ms/step (wall {wall:.1f} s)", file=sys.stderr, flush=True)
    value = pairs / (ms_step / 1e3)

    if a.copy_calib_mib:
        src = torch.ones(a.copy_calib_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # roofline of the dominant kernel (stage 1: seed + 3 conv/ReLU layers at 32x32 + pool)
    st1 = prof.get(f"myrtle_stage1_n{hw}")
    roof = None
    if st1:
        launches, tot_ms = st1
        launches_per_step = launches / done
        pairs_per_launch = pairs / launches_per_step
        flop_pair_st1 = (workmodel.FLOPS_PER_ENTRY_LAYER * depth[0] * hw ** 4
                         + workmodel.FLOPS_PER_SEED_ENTRY_PER_CHANNEL * 3 * hw ** 4
                         + workmodel.FLOPS_PER_POOLED_ENTRY * hw ** 4)
        avg_s = tot_ms / launches / 1e3
        achieved = flop_pair_st1 * pairs_per_launch / avg_s / 1e12
        traffic = _traffic(int(pairs_per_launch))
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic, "valu_counters": _valu_counters(), "kernel": f"myrtle_stage1_n{hw}",
                "avg_launch_ms": round(tot_ms / launches, 3), "pairs_per_launch": int(pairs_per_launch),
                "flops_per_pair": flop_pair_st1}
    flops_pair = workmodel.flops_per_pair(hw, 3, depth)
    rec.update({
        "value": round(value, 3), "steps": done, "warmup": warm, "ms_per_step": round(ms_step, 3),
        "ms_each_step": [round(v, 3) for v in ms_each], "ms_median_step": round(med, 3),
        "model_tflops_whole_step": round(flops_pair * pairs / (ms_step / 1e3) / 1e12, 3),
        "kernels_ms_per_step": {k: round(v[1] / done, 3) for k, v in prof.items()},
        "roofline": roof,
    })

    if not a.no_cpu_baseline:
        import oracle

        m = min(a.cpu_sample, n)
        cores = _host_threads()
        net = oracle.Myrtle(depth, w["sigma_w2"], w["sigma_b2"])
        pa, pb = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        plist = np.stack([pa.ravel(), pb.ravel()], 1)
        t = time.perf_counter()
        q1, d1 = oracle.myrtle_self(x1n[:m], net, cores)
        q2, d2 = oracle.myrtle_self(x2n[:m], net, cores)
        kr = oracle.myrtle_pairs(x1n[:m], x2n[:m], plist, net, q1, q2, cores).reshape(m, m)
        dt = time.perf_counter() - t
        rec["cpu_baseline"] = {
            "value": round(m * m / dt, 3), "unit": "entries/s", "cores": cores, "kind": "oracle",
            "per_core": round(m * m / dt / cores, 3),
            "sample": f"{m}x{m} sub-block of the same 4096x4096 Myrtle-10 block ({m * m} entries, plus "
                      f"{2 * m} self recursions for the variance maps; {dt:.1f} s of wall time, float64, "
                      f"{cores} OpenMP threads = the host cores given to this GPU)"}
        kg = out[:m, :m].cpu().numpy()
        err = float(np.max(np.abs(kg - kr) / np.sqrt(np.outer(d1, d2))))
        rec["parity"] = {"max_normalised_error": err, "entries": m * m, "tolerance": 2e-5}
        print(f"[{_elapsed():.1f} s] oracle sample: {dt:.1f} s, parity {err:.2e}", file=sys.stderr, flush=True)

    # Side legs, in order of importance, each with an estimate of its wall
    # time: a leg that would end past the budget is skipped by name.
    legs = [
        ("fwd_bwd", 20.0, a.no_fwd_bwd, lambda: _fwd_bwd(torch)),
        ("batched_tiles", 75.0, a.no_batched, lambda: _batched(torch, a.batched_full, a.batched_reps)),
        ("ntk", 12.0, a.no_ntk, lambda: _ntk(torch)),
        ("cv8", 15.0, a.no_cv8, lambda: _cv8(torch, not a.no_cpu_baseline)),
        ("myrtle7_64x64", 10.0, a.no_64, lambda: _myrtle64(torch)),
        ("pcg", 35.0, a.no_pcg, lambda: _pcg(torch, not a.no_cpu_baseline)),
        ("approx_solvers", 30.0, a.no_approx, lambda: _approx(torch)),
    ]
    for name, est, off, fn in legs:
        if off:
            rec[name] = None
            continue
        if _elapsed() + est > a.budget_s:
            rec[name] = {"skipped": "budget", "estimated_s": est, "elapsed_s": round(_elapsed(), 1)}
            print(f"[{_elapsed():.1f} s] {name}: skipped (budget)", file=sys.stderr, flush=True)
            continue
        t = time.perf_counter()
        res = fn()
        from paper_2303_05420_amd import ops as _ops
        _ops.release_workspace()  # (the fwd_bwd leg's workspace is large)
        torch.cuda.empty_cache()
        res["leg_wall_s"] = round(time.perf_counter() - t, 2)
        if name == "pcg":
            rec["fc3_gram"] = res.pop("fc_gram")
        rec[name] = res
        print(f"[{_elapsed():.1f} s] {name}: done in {res['leg_wall_s']} s", file=sys.stderr, flush=True)
    rec["wall_s"] = round(_elapsed(), 1)
    _emit(rec)


if __name__ == "__main__":
    main()
