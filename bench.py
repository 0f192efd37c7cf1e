"""Benchmark of the VQMC + SR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 10x10|16x16|24x24]
                    [--conv fp32|bf16|bf16x3] [--sr auto|chol32|chol64|dual|cg]

One step = local energies of B samples (every exchanged configuration
evaluated), per-sample log-derivatives O_k, and one SR solve
(S + eps I) delta = F, on inputs resident in GPU memory.  Prints one JSON
line.  The sampler that produces the 10x10 configurations (1000 sweeps from
the Neel state) runs before the timed region and is reported separately.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VQMC samples/s (E_loc+O_k+SR step) at 10×10 & 24×24, J2/J1=0.5; BF16 vs FP32"
PEAK = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "fp64": 78.6}  # TFLOP/s, dense
HBM_PEAK = 8000.0  # GB/s


def f_cfg(L, C, n):
    """Dense FLOPs of one configuration's forward pass (2 per multiply-add)."""
    return 2 * L * L * 9 * (C + n * C * C)


def antiparallel_counts(spins, L):
    """Antiparallel bonds per configuration, by bond kind (right, below,
    lower-right, lower-left): bench-side bookkeeping for FLOP counts."""
    s = spins.reshape(-1, L, L).astype(np.int16)
    return np.stack([(s != np.roll(s, (-dy, -dx), axis=(1, 2))).sum(axis=(1, 2))
                     for dy, dx in ((0, 1), (1, 0), (1, 1), (1, -1))], axis=1)


def eloc_flops(spins, L, C, n, lightcone, conv):
    """(algorithmic, executed) FLOPs of one local-energy call.

    Algorithmic: dense, (1 + n_ap) forward passes per sample; light cone, one
    forward pass per sample plus, per exchanged pair and layer, the
    convolution rows of the pair's neighbourhood at that distance.

    Executed: the products the matrix cores run in the convolution precision,
    counted as the kernels issue them.  Dense: every batch of up to G = rows /
    N configurations runs the 16-row tiles of the workgroup's four waves (448
    rows in the C = 16 BF16 forms at up to 448 sites, else 512 at C <= 16 and
    576 at C = 32; the BF16 forms skip a wave's last tile when it starts past
    the batch's rows), with K padded to whole instruction steps (4 for FP32,
    32 for BF16: 144 -> 160 at C = 16), plus, for FP32, the 1 -> C lift (K = 9
    padded to 12; in the BF16 forms the lift runs on the FP32 matrix cores
    and is not counted here).
    Light cone: the neighbourhood rows padded to 16-row tiles (the FP32 pass
    of the sampled configuration is counted only for the FP32 form).
    Split-BF16 runs three products per output."""
    nap = antiparallel_counts(spins, L)
    mult = 3 if conv == "bf16x3" else 1
    N = L * L
    B = spins.shape[0]
    if not lightcone:
        f = float((1 + nap.sum(axis=1)).sum()) * f_cfg(L, C, n)
        if conv == "fp32":
            kstep, rows = 4, 4 * (9 if C == 32 else 8) * 16
        else:
            kstep = 32
            rows = 4 * 7 * 16 if (C == 16 and N <= 448) else 4 * (9 if C == 32 else 8) * 16
        G = min(rows // N, 64)
        kpad = -(-9 * C // kstep) * kstep
        ntc = -(-C // 16) * 16
        tpw = rows // 64

        def tiles(r):  # tiles one batch of r rows runs
            if conv == "fp32":
                return 4 * tpw
            return 4 * (tpw - 1) + sum(1 for w in range(4) if (w + 4 * (tpw - 1)) * 16 < r)

        nconf = 1 + nap.sum(axis=1)
        nb = -(-nconf // G)
        last = nconf - G * (nb - 1)
        t = float((nb - 1).sum()) * tiles(G * N) + sum(float(c) * tiles(int(g) * N)
                                                        for g, c in zip(*np.unique(last, return_counts=True)))
        per_tile = 16 * ntc * 2 * (n * kpad + (12 if conv == "fp32" else 0))
        return f, t * per_tile * mult
    per_row = 2 * 9 * C * C
    alg = np.zeros(4)
    exe = np.zeros(4)
    for kind, (ey, ex) in enumerate(((0, 1), (1, 0), (1, 1), (1, 1))):
        for l in range(1, n + 1):
            d = l + 1
            rows = min(ey + 1 + 2 * d, L) * min(ex + 1 + 2 * d, L)
            alg[kind] += rows * per_row
            exe[kind] += -(-rows // 16) * 16 * per_row
    base = B * f_cfg(L, C, n)
    return base + float((nap * alg).sum()), (base if conv == "fp32" else 0.0) + float((nap * exe).sum()) * mult


WORKLOADS = {
    # S accumulated on the FP32 matrix cores is not positive definite at
    # eps = 1e-4 on the sampled O (the factorisation reports it), so the
    # explicit S is formed on the FP64 matrix cores; chol32 stays a variant
    "10x10": dict(L=10, C=16, n=6, B=4096, spins="sampled", sr="chol64"),
    "16x16": dict(L=16, C=32, n=8, B=8192, spins="uniform", sr="cg"),
    "24x24": dict(L=24, C=32, n=8, B=16384, spins="uniform", sr="cg"),
}


SR_NAMES = {"chol32": "Cholesky of S, S on FP32 matrix cores", "chol64": "Cholesky of S, S in FP64",
            "dual": "Cholesky of the B x B sample-space matrix, FP64", "cg": "CG, tol 1e-8, at most 200 iterations"}


def sr_opts(V, name):
    return {
        "chol32": V.SrOpts(method=V.SR_CHOLESKY, s_prec=0, eps=1e-4),
        "chol64": V.SrOpts(method=V.SR_CHOLESKY, s_prec=1, eps=1e-4),
        "dual": V.SrOpts(method=V.SR_DUAL, eps=1e-4),
        "cg": V.SrOpts(method=V.SR_CG, eps=1e-4, tol=1e-8, max_iter=200),
    }[name]


def sr_stage_roofline(sr_name, B, P, ms, iters):
    """The whole SR stage against the roofline of its arithmetic, from the
    stage's event time: the explicit S (B P^2 FLOPs for its lower half) plus
    the Cholesky (P^3 / 3) and the two triangular solves (2 P^2); the
    sample-space form (B^2 P for the Gram matrix, B^3 / 3, two passes over O);
    CG by its HBM bytes (two passes over O per iteration)."""
    t = ms / 1e3
    if sr_name in ("chol32", "chol64"):
        flops = B * P * P + P ** 3 / 3 + 2 * P * P
        scope = "S (B P^2) + Cholesky (P^3/3) + solves (2 P^2) FLOPs over the SR stage time"
    elif sr_name == "dual":
        flops = B * B * P + B ** 3 / 3 + 4 * B * P
        scope = "Gram matrix (B^2 P) + Cholesky (B^3/3) + two passes over O FLOPs over the SR stage time"
    else:
        gbs = 2 * B * P * 4 * iters / t / 1e9
        return {"bound": "hbm", "scope": "two passes over O per CG iteration over the SR stage time",
                "achieved": gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": gbs / HBM_PEAK}
    tf = flops / t / 1e12
    return {"bound": "mfma", "scope": scope, "flops": flops, "achieved": tf, "peak": PEAK["fp64"],
            "unit": "TFLOP/s", "frac": tf / PEAK["fp64"]}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, th, spins, sample):
    """The FP64 oracle on a bounded sample of the same workload."""
    import oracle as R
    m = R.RefModel(wl["L"], wl["C"], wl["n"], 1.0, 0.5, 1)
    s = spins[:sample]
    t0 = time.perf_counter()
    e = R.local_energy(m, th, s)
    O = R.log_derivs(m, th, s)
    R.sr_solve(O, e, 1e-4)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sample / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "first %d of the %d configurations: E_loc + O_k + exact SR solve on that "
                      "subset, FP64 plain loops (%.1f s)" % (sample, len(spins), dt)}


def cpu_extra():
    """Oracle timings of the SR algebra at full size (host-memory bound; a
    few minutes of CPU): the exact 10x10 solve by both exact forms on a
    seeded O (B = 4096, P = 14080), and one application of S + eps I at
    24x24 (B = 16384, P = 74304), the work of one CG iteration."""
    import oracle as R
    out = {"cpu_model": cpu_model(), "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
    rng = np.random.default_rng(3)
    B, P = 4096, 14080
    O = rng.standard_normal((B, P)) * 0.1
    E = rng.standard_normal(B) - 50
    for name, method in (("sample_space", 1), ("explicit_S", 0)):
        t0 = time.perf_counter()
        R.sr_solve(O, E, 1e-4, method=method)
        out["sr_10x10_" + name + "_s"] = time.perf_counter() - t0
        print(json.dumps({"cpu_extra": name, "s": out["sr_10x10_" + name + "_s"]}), flush=True)
    del O
    B, P = 16384, 74304
    O = np.full((B, P), 0.5)
    mean = O.mean(axis=0)
    v = np.ones(P)
    t0 = time.perf_counter()
    R.sr_apply(O, mean, v, 1e-4)
    out["sr_apply_24x24_s"] = time.perf_counter() - t0
    out["sr_apply_24x24_gbs"] = 2 * B * P * 8 / out["sr_apply_24x24_s"] / 1e9
    return out


TRAFFIC_RECORDS = os.path.join(ROOT, "profiles", "hbm_traffic.md")
KERNEL_SOURCES = {
    "eloc_kernel": ["forward.hip", "engine.hpp", "common.hpp"],
    "eloc_lc_kernel": ["eloc_lc.hip", "eloc_lc.hpp", "engine.hpp", "common.hpp"],
}


def sources_digest(kernel):
    """SHA-256 over the sources a kernel is compiled from, so that a stored
    counter reading is only used for the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2108_13830_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel, workload_key):
    """HBM bytes per launch of `kernel` on this workload from the counter
    table (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factors), or
    None when there is no reading or the kernel changed since it was taken.
    Table rows: | kernel | workload | sources sha256 | bytes per launch | ..."""
    if not os.path.exists(TRAFFIC_RECORDS):
        return None
    digest = sources_digest(kernel)
    for line in open(TRAFFIC_RECORDS):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == kernel and cells[1] == workload_key and cells[2] == digest:
            return float(cells[3])
    return None


def copy_calibration(mib):
    """A streaming elementwise kernel over `mib` MiB in and out (torch.neg on
    float32): the kernel of known traffic that scales the HBM byte counters."""
    import torch
    nel = mib << 18
    x = torch.ones(nel, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "torch.neg float32", "bytes_in": nel * 4,
                                           "bytes_out": nel * 4, "launches": 3}}), flush=True)


def measured_ceilings(V, torch):
    """What this GPU sustains: matrix-instruction loops per kind (the
    library's probe, register operands only) and a streaming copy of 1 GiB
    in and 1 GiB out (torch.neg on float32), timed with HIP events."""
    c = {"mfma_tflops": {"bf16": V.probe_mfma("bf16", iters=400, blocks=1024),
                         "fp32": V.probe_mfma("fp32", iters=400, blocks=1024),
                         "fp64": V.probe_mfma("fp64", iters=200, blocks=1024)}}
    nel = 1 << 28
    x = torch.ones(nel, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.neg(x, out=y)
    e1.record()
    torch.cuda.synchronize()
    c["copy_gbs"] = 5 * 2 * nel * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    return c


def other_workload(V, torch, name, convs):
    """One full step of another workload (uniform Sz = 0 configurations) per
    convolution form: samples/s and stage times, for the other lattices the
    metric names.  One warm-up step, one timed step per form; then the exact
    sample-space solve of each form's system, timed once, beside CG, and the
    distance of the CG solution from it."""
    from vqmc_inputs import init_theta, uniform_sz0
    wl = WORKLOADS[name]
    L, C, n, B = wl["L"], wl["C"], wl["n"], wl["B"]
    dev = torch.device("cuda:0")
    th = torch.from_numpy(init_theta(C, n, seed=0)).to(dev)
    spins = torch.from_numpy(uniform_sz0(L, B, seed=1)).to(dev)
    spins_np = spins.cpu().numpy()
    res = {"workload": "%s periodic J1-J2 (J2/J1=0.5), C=%d, n=%d, B=%d uniform Sz=0 configurations; "
                       "E_loc (light cone) + O_k + SR (%s)" % (name, C, n, B, SR_NAMES[wl["sr"]])}
    base = V.Model(L, C, n, 1.0, 0.5, 1, V.PREC_FP32, V.ELOC_AUTO)
    P = V.num_params(base)
    O = torch.empty((B, P), dtype=torch.float32, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    ws_o = torch.empty(max(V.log_derivs_workspace(base, B), 1), dtype=torch.uint8, device=dev)
    opts = sr_opts(V, wl["sr"])
    ws_sr = torch.empty(max(V.sr_workspace(B, P, opts), 1), dtype=torch.uint8, device=dev)
    exact = sr_opts(V, "dual")
    ws_x = torch.empty(max(V.sr_workspace(B, P, exact), 1), dtype=torch.uint8, device=dev)
    delta = torch.empty(P, dtype=torch.float64, device=dev)
    dx = torch.empty(P, dtype=torch.float64, device=dev)
    for conv in convs:
        gm = base.with_prec(conv)
        lightcone = V.local_energy_method(gm) == V.ELOC_LIGHTCONE
        nb = V.local_energy_workspace(gm, B)
        ws_e = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None
        for it in range(2):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev[0].record()
            V.vqmc_local_energy(gm, th, spins, out=e, workspace=ws_e)
            ev[1].record()
            V.vqmc_log_derivs(base, th, spins, O=O, workspace=ws_o)
            ev[2].record()
            _, _, info = V.vqmc_sr_solve(O, e, opts, delta=delta, workspace=ws_sr)
            ev[3].record()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        st = [ev[j].elapsed_time(ev[j + 1]) for j in range(3)]
        fa, fe = eloc_flops(spins_np, L, C, n, lightcone, conv)
        r = {"samples_per_s": B / wall, "ms_per_step": wall * 1e3,
             "stage_ms": {"local_energy": st[0], "log_derivs": st[1], "sr_solve": st[2]},
             "eloc": "lightcone" if lightcone else "dense",
             "eloc_tflops_algorithmic": fa / (st[0] / 1e3) / 1e12,
             "eloc_tflops_executed": fe / (st[0] / 1e3) / 1e12,
             "eloc_executed_frac_of_peak": fe / (st[0] / 1e3) / 1e12 / PEAK[conv]}
        if wl["sr"] == "cg":
            r.update({"cg_iterations": info["iters"], "cg_rel_residual": info["rel_residual"],
                      "cg_hbm_gbs": info["iters"] * 2 * B * P * 4 / (st[2] / 1e3) / 1e9})
        # the exact solution of the same system (sample-space Cholesky, FP64)
        evx = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        evx[0].record()
        V.vqmc_sr_solve(O, e, exact, delta=dx, workspace=ws_x, want_info=False)
        evx[1].record()
        torch.cuda.synchronize()
        r["delta_rel_err_vs_exact"] = (torch.linalg.vector_norm(delta - dx) / torch.linalg.vector_norm(dx)).item()
        if "sr_exact" not in res:
            ms = evx[0].elapsed_time(evx[1])
            # lower half of the B x B Gram matrix: B^2 P FLOPs on the FP64 matrix cores
            res["sr_exact"] = {"form": SR_NAMES["dual"], "sr_solve_ms_first_call": ms,
                               "gram_tflop": B * B * P / 1e12}
        res[conv] = r
        del ws_e
    # the exact solve timed on its own, warm
    evx = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    evx[0].record()
    V.vqmc_sr_solve(O, e, exact, delta=dx, workspace=ws_x, want_info=False)
    evx[1].record()
    torch.cuda.synchronize()
    ms = evx[0].elapsed_time(evx[1])
    res["sr_exact"].update({"sr_solve_ms": ms, "gram_tflops": B * B * P / (ms / 1e3) / 1e12,
                            "samples_per_s_with_exact_sr": {
                                c: B / ((res[c]["stage_ms"]["local_energy"] + res[c]["stage_ms"]["log_derivs"]
                                         + ms) / 1e3) for c in convs}})
    del ws_sr, ws_x
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="10x10", choices=sorted(WORKLOADS))
    ap.add_argument("--conv", default="fp32", choices=["fp32", "bf16", "bf16x3"])
    ap.add_argument("--sr", default=None, choices=["chol32", "chol64", "dual", "cg"])
    ap.add_argument("--eloc", default="auto", choices=["auto", "dense", "lightcone"])
    ap.add_argument("--samples", type=int, default=None, help="override B")
    ap.add_argument("--burn-in", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="bf16x3,bf16,chol32,dual,sym",
                    help="extra forms timed on the same inputs (comma list, or 'none')")
    ap.add_argument("--also", default="24x24,16x16",
                    help="other workloads timed after the main one (one step per form, bf16x3, bf16 and fp32; "
                         "comma list), or 'none'")
    ap.add_argument("--cpu-extra", action="store_true",
                    help="only time the oracle's full-size SR algebra on the host (minutes), then exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the copy kernel that scales HBM byte counters, then exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.cpu_extra:
        print(json.dumps({"cpu_extra": cpu_extra()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: libvqmc has no multi-GPU path "
              "(samples would shard across GPUs with one all-reduce per SR step); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2108_13830_amd import vqmc as V
    from vqmc_inputs import init_theta, neel, uniform_sz0

    wl = dict(WORKLOADS[args.workload])
    if args.samples:
        wl["B"] = args.samples
    sr_name = args.sr or wl["sr"]
    L, C, n, B = wl["L"], wl["C"], wl["n"], wl["B"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    th_np = init_theta(C, n, seed=0)
    th = torch.from_numpy(th_np).to(dev)
    eloc_mode = {"auto": V.ELOC_AUTO, "dense": V.ELOC_DENSE, "lightcone": V.ELOC_LIGHTCONE}[args.eloc]
    gm = V.Model(L, C, n, 1.0, 0.5, 1, V.PREC_NAMES[args.conv], eloc_mode)
    lightcone = V.local_energy_method(gm) == V.ELOC_LIGHTCONE
    P = V.num_params(gm)

    # ---- inputs (resident before the timed region)
    sampler = None
    if wl["spins"] == "sampled":
        spins = torch.from_numpy(neel(L, B)).to(dev)
        acc = torch.empty(B, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V.vqmc_sample(gm.with_prec("fp32"), th, spins, n_sweeps=args.burn_in, seed=2, n_accepted=acc)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        sampler = {"chains": B, "sweeps": args.burn_in, "seconds": ts,
                   "proposals_per_s": B * args.burn_in * L * L / ts,
                   "acceptance": float(acc.sum().item()) / (B * args.burn_in * L * L)}
    else:
        spins = torch.from_numpy(uniform_sz0(L, B, seed=1)).to(dev)
    spins_np = spins.cpu().numpy()
    e = torch.empty(B, dtype=torch.float64, device=dev)
    O = torch.empty((B, P), dtype=torch.float32, device=dev)
    ws_o = torch.empty(max(V.log_derivs_workspace(gm, B), 1), dtype=torch.uint8, device=dev)
    ws_e = {}

    def eloc_ws(model):
        if model not in ws_e:
            nb = V.local_energy_workspace(model, B)
            ws_e[model] = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None
        return ws_e[model]
    opts = sr_opts(V, sr_name)
    ws_sr = torch.empty(max(V.sr_workspace(B, P, opts), 1), dtype=torch.uint8, device=dev)
    delta = torch.empty(P, dtype=torch.float64, device=dev)
    F = torch.empty(P, dtype=torch.float64, device=dev)

    def run_step(model, o, ws, times=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if times is not None else None
        if ev:
            ev[0].record()
        V.vqmc_local_energy(model, th, spins, out=e, workspace=eloc_ws(model))
        if ev:
            ev[1].record()
        V.vqmc_log_derivs(model.with_prec("fp32"), th, spins, O=O, workspace=ws_o)
        if ev:
            ev[2].record()
        V.vqmc_sr_solve(O, e, o, delta=delta, F=F, workspace=ws, want_info=False)
        if ev:
            ev[3].record()
            times.append(ev)

    def timed(model, o, ws, steps, warmup):
        for _ in range(warmup):
            run_step(model, o, ws)
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            run_step(model, o, ws, evs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = np.array([[evs[i][j].elapsed_time(evs[i][j + 1]) for j in range(3)] for i in range(steps)])
        return wall / steps * 1e3, st.mean(axis=0)

    ms, stage = timed(gm, opts, ws_sr, args.steps, args.warmup)
    value = B / (ms / 1e3)
    # after the timed region: the solve's report on the same inputs, and the
    # distance of its delta from the exact FP64 sample-space solution of the
    # same system (the reference every SR form is measured against here)
    d_main = delta.clone()

    def sr_status(o, ws):
        """The solve's own report (status, CG iterations and residual) on the
        current O and E, run once with info after the timed steps."""
        try:
            _, _, info = V.vqmc_sr_solve(O, e, o, delta=delta, F=F, workspace=ws)
            info["status"] = "ok" if info["converged"] else V.STATUS[V.WARN_NOT_CONVERGED]
        except V.VqmcError as err:
            info = {"status": V.STATUS.get(err.status, str(err.status)), "iters": 0,
                    "rel_residual": float("nan")}
        return info
    sr_info = sr_status(opts, ws_sr)
    exact = sr_opts(V, "dual")
    ws_x = torch.empty(max(V.sr_workspace(B, P, exact), 1), dtype=torch.uint8, device=dev)
    d_exact = torch.empty(P, dtype=torch.float64, device=dev)
    V.vqmc_sr_solve(O, e, exact, delta=d_exact, workspace=ws_x, want_info=False)
    del ws_x

    def delta_err(d):
        return (torch.linalg.vector_norm(d - d_exact) / torch.linalg.vector_norm(d_exact)).item()

    # ---- roofline of the dominant kernel (the fused local-energy kernel:
    # one launch per call, so the call's event time is the kernel's time)
    flops_eloc, flops_exec = eloc_flops(spins_np, L, C, n, lightcone, args.conv)
    dense_equiv, _ = eloc_flops(spins_np, L, C, n, False, args.conv)
    t_eloc = stage[0] / 1e3
    conv_peak = PEAK[args.conv]
    achieved = flops_eloc / t_eloc / 1e12
    kname = "eloc_lc_kernel" if lightcone else "eloc_kernel"
    wkey = "%s %s %s B=%d" % (args.workload, args.conv, "lightcone" if lightcone else "dense", B)
    roof = {"bound": "mfma", "kernel": kname,
            "achieved": achieved, "peak": conv_peak, "unit": "TFLOP/s", "frac": achieved / conv_peak,
            "traffic": stored_traffic(kname, wkey), "traffic_workload": wkey,
            "algorithmic_flops_per_launch": flops_eloc,
            "executed_mfma_flops_per_launch": flops_exec,
            "executed_tflops": flops_exec / t_eloc / 1e12,
            "dense_equivalent_tflops": dense_equiv / t_eloc / 1e12}

    ceil = measured_ceilings(V, torch)
    ach_peak = ceil["mfma_tflops"]["bf16" if args.conv != "fp32" else "fp32"]
    roof["achievable_peak"] = ach_peak
    roof["frac_of_achievable"] = achieved / ach_peak

    out = {"metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.conv, "data": "synthetic",
           "config": {"workload": "%s periodic J1-J2 (J2/J1=0.5), C=%d, n=%d, P=%d, B=%d %s configurations; "
                                  "E_loc (%s) + O_k + SR (%s), %s convolutions"
                                  % (args.workload, C, n, P, B, wl["spins"],
                                     "light cone" if lightcone else "dense", sr_name, args.conv),
                      "L": L, "channels": C, "layers": n, "params": P, "samples": B,
                      "conv": args.conv, "sr": sr_name, "eloc": "lightcone" if lightcone else "dense"},
           "stage_ms": {"local_energy": stage[0], "log_derivs": stage[1], "sr_solve": stage[2]},
           "sr_report": {"status": sr_info["status"],
                         "iters": sr_info["iters"], "rel_residual": sr_info["rel_residual"],
                         "delta_rel_err": delta_err(d_main),
                         "delta_reference": "sample-space Cholesky, FP64, same O and E",
                         "delta_bar": 1e-3, "meets_delta_bar": delta_err(d_main) <= 1e-3},
           "roofline": roof,
           "sr_roofline": sr_stage_roofline(sr_name, B, P, stage[2], sr_info["iters"]),
           "measured_ceilings": ceil}
    if sampler:
        out["sampler"] = sampler

    variants = {}
    if args.variants != "none":
        for v in args.variants.split(","):
            if v in ("bf16", "bf16x3", "fp32") and v != args.conv:
                vms, vst = timed(gm.with_prec(v), opts, ws_sr, 1, 1)
                lc_v = V.local_energy_method(gm.with_prec(v)) == V.ELOC_LIGHTCONE
                _, fe_v = eloc_flops(spins_np, L, C, n, lc_v, v)
                variants["conv_" + v] = {"samples_per_s": B / (vms / 1e3), "ms_per_step": vms,
                                         "stage_ms": vst.tolist(),
                                         "eloc_tflops_algorithmic": flops_eloc / (vst[0] / 1e3) / 1e12,
                                         "eloc_tflops_executed": fe_v / (vst[0] / 1e3) / 1e12,
                                         "eloc_executed_frac_of_peak": fe_v / (vst[0] / 1e3) / 1e12 / PEAK[v],
                                         "delta_rel_err": delta_err(delta)}
            elif v in ("dense", "lightcone"):
                vm = gm.with_eloc(V.ELOC_DENSE if v == "dense" else V.ELOC_LIGHTCONE)
                if (v == "lightcone") == lightcone:
                    continue
                vms, vst = timed(vm, opts, ws_sr, 1, 1)
                fa, _ = eloc_flops(spins_np, L, C, n, v == "lightcone", args.conv)
                variants["eloc_" + v] = {"samples_per_s": B / (vms / 1e3), "ms_per_step": vms,
                                         "stage_ms": vst.tolist(),
                                         "eloc_tflops_algorithmic": fa / (vst[0] / 1e3) / 1e12}
            elif v == "sym":
                # the rotation-symmetrised amplitude: four turned configurations
                # per sample in E_loc and O_k (same SR)
                vms, vst = timed(gm.with_symmetry(1), opts, ws_sr, 1, 1)
                variants["sym"] = {"samples_per_s": B / (vms / 1e3), "ms_per_step": vms,
                                   "stage_ms": vst.tolist(),
                                   "eloc_tflops_algorithmic": 4 * flops_eloc / (vst[0] / 1e3) / 1e12}
            elif v in ("chol32", "chol64", "dual", "cg") and v != sr_name:
                vo = sr_opts(V, v)
                vws = torch.empty(max(V.sr_workspace(B, P, vo), 1), dtype=torch.uint8, device=dev)
                vms, vst = timed(gm, vo, vws, 1, 1)
                variants["sr_" + v] = {"samples_per_s": B / (vms / 1e3), "ms_per_step": vms,
                                       "stage_ms": vst.tolist(), "delta_rel_err": delta_err(delta),
                                       "sr_status": sr_status(vo, vws)["status"]}
                del vws
    if variants:
        out["variants"] = variants
    also = [w for w in args.also.split(",") if w not in ("none", "", args.workload)]
    if also:
        del O, ws_o, ws_sr, ws_e
        torch.cuda.empty_cache()
        out["also"] = {}
        for w in also:
            out["also"][w] = other_workload(V, torch, w, ["bf16x3", "bf16", "fp32"])
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, th_np, spins_np, min(args.cpu_sample, B))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
