"""Benchmark of the scattering self-energy forward on one MI355X.

Workload: the device-scale electron-phonon problem (one GPU's share of a
~5k-atom FinFET slice): Nkz=Nqz=7, NE=1024, Nw=10, Na=4864, Nb=4, Norb=10,
complex128, G stored diagonal-only.  Inputs are seeded synthetic data drawn
on the GPU (see paper_1912_10024_amd/inputs.py); they are resident in HBM
before the timed region.  One step = one sse_forward call (one of
Sigma^< / Sigma^>), i.e. every stage of the hot path over the whole input.

Prints one JSON line (rank 0).  `value` is effective TFLOP/s, the paper's
regrouped-form flop count (f_eff) divided by the time per step.  The line
also carries the phonon self-energy Pi (Eq. 4) on the same workload (Gs = G<,
Go = G>), timed the same way, under "phonon", and the adjoint's three
gradients on the mid workload under "adjoint".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK = 78.6e12   # MI355X dense fp64 matrix peak, flop/s
FP32_MFMA_PEAK = 157.3e12
FP16_MFMA_PEAK = 2.5e15    # dense fp16 matrix peak
HBM_PEAK = 8.0e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="device", choices=["tiny", "mid", "device", "mid12", "direct5"],
                   help="workload; mid12: the mid workload with 12 orbitals (the paper's count), fp64 and fp32 "
                        "forms only, with --no-phonon --no-adjoint; direct5: 1024 atoms, NE 64 with 5 "
                        "neighbours (no matrix-core instance: the direct fp64 kernel), fp64 only, with "
                        "--no-phonon --no-adjoint")
    p.add_argument("--forms", default="fp64,fp32,bf16x2,fp16x2,fp16",
                   help="comma-separated operand precisions to time; the first is the headline value "
                        "(fp16 and fp16_unscaled: the single-term comparison forms)")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-phonon", action="store_true", help="skip the phonon self-energy timing")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing (mid workload)")
    p.add_argument("--only-phonon", action="store_true", help="time only the phonon self-energy (profiling runs)")
    p.add_argument("--only-adjoint", action="store_true",
                   help="time only the adjoint on the mid workload and its forward (profiling runs)")
    p.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                   help="only run a plain device copy of this many GiB (scales HBM byte counters)")
    return p.parse_args()


def compact_problem(d, G, D, dH, nbr, atoms):
    """Host copy of everything the outputs of `atoms` depend on, with atoms renumbered."""
    import torch
    from paper_1912_10024_amd.inputs import Dims

    nbr_h = nbr.cpu().numpy()
    keep = sorted(set(int(a) for a in atoms) | set(int(b) for a in atoms for b in nbr_h[a]))
    remap = {a: i for i, a in enumerate(keep)}
    idx = torch.tensor(keep, device=G.device)
    sub = Dims(nkz=d.nkz, ne=d.ne, nqz=d.nqz, nw=d.nw, na=len(keep), nb=d.nb, norb=d.norb, g_slots=1)
    Gs = G[:, :, :, :1].index_select(2, idx).cpu().numpy()
    Ds = D.index_select(2, idx).cpu().numpy()
    Hs = dH.index_select(0, idx).cpu().numpy()
    # atoms outside `atoms` keep a valid (unused) neighbour row: point at themselves' first kept atom
    nb_s = np.zeros((len(keep), d.nb), dtype=np.int32)
    for a in keep:
        if a in set(int(x) for x in atoms):
            nb_s[remap[a]] = [remap[int(b)] for b in nbr_h[a]]
        else:
            nb_s[remap[a]] = [(remap[a] + 1 + t) % len(keep) for t in range(d.nb)]
    return sub, np.ascontiguousarray(Gs), np.ascontiguousarray(Ds), np.ascontiguousarray(Hs), nb_s, remap


def cpu_baseline(d, G, D, dH, nbr, target_s, f_block, seed=7):
    """Time the CPU oracle on a bounded sample of output blocks of this workload.
    Returns the baseline record, the sampled (k, E, a) blocks and their values,
    which every GPU form is checked against."""
    from oracle import oracle

    rng = np.random.default_rng(seed)
    atoms = rng.choice(d.na, size=4, replace=False)
    sub, Gs, Ds, Hs, nbs, remap = compact_problem(d, G, D, dH, nbr, atoms)
    oracle.num_threads()

    def pts_for(n):
        ks = rng.integers(d.nkz, size=n)
        es = rng.integers(d.ne, size=n)
        aa = rng.choice(atoms, size=n)
        return [(int(k), int(e), int(a)) for k, e, a in zip(ks, es, aa)]

    # calibrate on enough blocks to keep every host thread busy (a short
    # calibration overestimates the per-block time), then run a sample sized
    # to target_s
    oracle.sse_points(sub, Gs, Ds, Hs, nbs, [(k, e, remap[a]) for k, e, a in pts_for(32)])  # warm-up
    cal = pts_for(512)
    t0 = time.perf_counter()
    oracle.sse_points(sub, Gs, Ds, Hs, nbs, [(k, e, remap[a]) for k, e, a in cal])
    per = (time.perf_counter() - t0) / len(cal)
    n = int(max(16, min(200000, target_s / max(per, 1e-6))))
    pts = pts_for(n)
    t0 = time.perf_counter()
    ref = oracle.sse_points(sub, Gs, Ds, Hs, nbs, [(k, e, remap[a]) for k, e, a in pts])
    t = time.perf_counter() - t0
    return {
        "value": n * f_block / t / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{n} output blocks Sigma[kz,E,a] of the same workload (4 seeded atoms, random kz and E), {t:.1f} s",
        "seconds": t,
    }, pts, ref


def sampled_error(S, pts, ref):
    import torch

    idx = torch.tensor(pts, device=S.device)
    got = S[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def phonon_sample_error(d, Gs, Go, dH, nbr, P, seed=11):
    """Relative error of sampled Pi blocks against the CPU oracle.  Part of the
    CPU-oracle leg: it runs only with the CPU baseline (not with --no-cpu)."""
    import torch
    from oracle import oracle
    from paper_1912_10024_amd.inputs import Dims

    rng = np.random.default_rng(seed)
    atoms = [int(x) for x in rng.choice(d.na, size=2, replace=False)]
    # the Pi blocks of an atom read Gs at the atom, Go at its neighbours and its grad H
    nbr_h = nbr.cpu().numpy()
    keep = sorted(set(atoms) | set(int(b) for a in atoms for b in nbr_h[a]))
    remap = {a: i for i, a in enumerate(keep)}
    idx = torch.tensor(keep, device=Gs.device)
    sub = Dims(nkz=d.nkz, ne=d.ne, nqz=d.nqz, nw=d.nw, na=len(keep), nb=d.nb, norb=d.norb, g_slots=1)
    Gs_h = np.ascontiguousarray(Gs[:, :, :, :1].index_select(2, idx).cpu().numpy())
    Go_h = np.ascontiguousarray(Go[:, :, :, :1].index_select(2, idx).cpu().numpy())
    Hs = np.ascontiguousarray(dH.index_select(0, idx).cpu().numpy())
    nbs = np.array([[remap[int(b)] for b in nbr_h[a]] if a in atoms else [(remap[a] + 1 + t) % len(keep)
                                                                          for t in range(d.nb)] for a in keep],
                   dtype=np.int32)
    pts = [(int(rng.integers(d.nqz)), int(rng.integers(d.nw)), a, int(rng.integers(d.nb))) for a in atoms for _ in range(3)]
    ref = oracle.pse_points(sub, Gs_h, Go_h, Hs, nbs, [(q, w, remap[a], n) for q, w, a, n in pts])
    pidx = torch.tensor(pts, device=P.device)
    got = P[pidx[:, 0], pidx[:, 1], pidx[:, 2], pidx[:, 3]].cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def kernel_source_hash(sources) -> str:
    """sha256 over the files a kernel is compiled from (in the given order)."""
    import hashlib

    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1912_10024_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


FWD_SOURCES = ("fwd_mfma.hip", "fwd_common.h", "sse_common.h")
H16_SOURCES = ("fwd_h16.hip", "fwd_common.h", "sse_common.h")
PSE_SOURCES = ("pse.hip", "sse_common.h")
BWD_SOURCES = ("bwd_mfma.hip", "sse_common.h")


def recorded_traffic(record, sources):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counters,
    if the kernel's sources are unchanged since they were taken."""
    rec = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(rec):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(rec) if "=" in l and not l.startswith("#"))
    if kv.get("kernel_source_sha256") != kernel_source_hash(sources):
        return None
    return float(kv["fetch_bytes"]) + float(kv["write_bytes"])


def fwd_mfma_dispatches(d, dev) -> int:
    """Kernel dispatches of one fp64 / fp32 forward call: the atoms go in batches
    of about twelve rounds of workgroups (12 * compute units / Norb, a multiple of
    8), as launch_fwd_flags in fwd_mfma.hip issues them."""
    import torch

    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    batch = max(8, 12 * cus // d.norb // 8 * 8)
    na8 = (d.na + 7) // 8 * 8
    return (na8 + batch - 1) // batch


def time_form(sse, G, D, dH, nbr, S, ws, form, steps, warmup, dev):
    import torch

    for _ in range(warmup):
        sse.forward(G, D, dH, nbr, precision=form, out=S, ws=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        sse.forward(G, D, dH, nbr, precision=form, out=S, ws=ws)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def time_phonon(sse, Gs, Go, dH, nbr, d, P, steps, warmup, dev):
    import torch

    for _ in range(warmup):
        sse.phonon_forward(Gs, Go, dH, nbr, d.nqz, d.nw, out=P)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        sse.phonon_forward(Gs, Go, dH, nbr, d.nqz, d.nw, out=P)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def phonon_record(args, sse, flops, d, G, dH, nbr, dev):
    """Time Pi< = Eq. 4 with Gs = G<, Go = G> on the same workload."""
    import torch
    from paper_1912_10024_amd.inputs import CONFIG_INDEX, generate_device

    Go = generate_device(d, CONFIG_INDEX[args.config], device=dev, which=("G>",))["G>"]
    P = torch.empty(d.d_shape, dtype=torch.complex128, device=dev)
    wall, kern_ms = time_phonon(sse, G, Go, dH, nbr, d, P, args.steps, args.warmup, dev)
    ms = float(np.mean(kern_ms))
    useful = flops.pse_flops(d)
    rec = {
        "workload": f"electron-phonon SSE Pi^< forward ({args.config}), Gs = G<, Go = G>",
        "value": round(useful / (ms * 1e-3) / 1e12, 3),
        "unit": "TFLOP/s",
        "kernel_ms": round(ms, 3),
        "kernel_ms_all": [round(x, 3) for x in kern_ms],
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "roofline": {"bound": "mfma", "achieved": round(useful / (ms * 1e-3) / 1e12, 3),
                     "peak": FP64_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": round(useful / (ms * 1e-3) / FP64_MFMA_PEAK, 4),
                     "traffic": (recorded_traffic("pse_mfma_device_traffic.txt", PSE_SOURCES)
                                 if args.config == "device" else None),
                     "flops_per_launch": useful,
                     "what": "useful fp64 flops: the trace contraction on the matrix cores plus T = gradH.Go.gradH^H "
                             "on the vector ALUs (same fp64 peak)"},
    }
    if not args.no_cpu:
        rec["rel_err_vs_oracle_sampled"] = phonon_sample_error(d, G, Go, dH, nbr, P)
    del Go, P
    torch.cuda.empty_cache()
    return rec


def adjoint_record(args, sse, dev):
    """All three gradients of the hand-written adjoint (dG, dD, d gradH) on the
    mid workload, the size the differentiation form is specified on, next to
    the forward of the same size; HIP events on the current stream."""
    import torch
    from paper_1912_10024_amd.inputs import CONFIGS, CONFIG_INDEX, generate_device

    d = CONFIGS["mid"]
    inp = generate_device(d, CONFIG_INDEX["mid"], device=dev, which=("nbr", "G<", "D<", "dH", "W"))
    G, D, dH, nbr = inp["G<"], inp["D<"], inp["dH"], inp["nbr"]
    gS = inp["W"].conj().transpose(-1, -2).contiguous()   # dL/dSigma for L = Re sum tr(W Sigma)
    ws = sse.workspace(d, backward=True, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(max(args.steps, 1)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return out

    S = torch.empty(d.sigma_shape, dtype=torch.complex128, device=dev)
    fwd = timed(lambda: sse.forward(G, D, dH, nbr, out=S))
    bwd = timed(lambda: sse.backward(G, D, dH, nbr, gS, ws=ws))
    # dG and d gradH alone: the matrix-core dG / d gradH kernel (plus the reverse
    # adjacency and the share reduction, together under 0.1% of it)
    dgdh = timed(lambda: sse.backward(G, D, dH, nbr, gS, need=(True, False, True), ws=ws))
    del inp, G, D, dH, nbr, gS, S, ws
    torch.cuda.empty_cache()
    from paper_1912_10024_amd.flops import adjoint_dgdh_flops

    flops = adjoint_dgdh_flops(d)
    ms = float(np.mean(dgdh))
    achieved = flops / (ms * 1e-3) / 1e12
    return {"workload": "adjoint dL/dG, dL/dD, dL/d gradH of L = Re sum tr(W Sigma<) (mid: Nkz=7, NE=256, "
                        "Nqz=7, Nw=10, Na=1024, Nb=4, Norb=10)",
            "ms_all_gradients": round(float(np.mean(bwd)), 3), "ms_all": [round(x, 3) for x in bwd],
            "forward_ms": round(float(np.mean(fwd)), 3),
            "ratio_to_forward": round(float(np.mean(bwd)) / float(np.mean(fwd)), 2),
            "ms_dg_dgradh": round(ms, 3),
            "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK / 1e12,
                         "unit": "TFLOP/s", "frac": round(achieved * 1e12 / FP64_MFMA_PEAK, 4),
                         "traffic": recorded_traffic("bwd_mfma_mid_traffic.txt", BWD_SOURCES),
                         "flops_per_launch": flops,
                         "what": "useful fp64 flops of the dG / d gradH kernel: Y = conj(alpha D) . W on the matrix "
                                 "cores and the 27 block products built on it (flops.adjoint_dgdh_flops)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the self-energy kernels run on one GPU per process; there is no multi-GPU path "
                                   "(the sharding design is in the design notes)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n}), flush=True)
        return

    from paper_1912_10024_amd import flops, sse
    from paper_1912_10024_amd.inputs import CONFIGS, CONFIG_INDEX, generate_device

    if args.config == "mid12":
        # the Norb = 12 instance of the matrix-core forward: the mid sizes with 12
        # orbitals (inputs drawn from the mid workload's streams)
        from paper_1912_10024_amd.inputs import Dims

        CONFIGS = dict(CONFIGS, mid12=Dims(nkz=7, ne=256, nqz=7, nw=10, na=1024, nb=4, norb=12, g_slots=1))
        CONFIG_INDEX = dict(CONFIG_INDEX, mid12=CONFIG_INDEX["mid"])
        bad = [f for f in args.forms.split(",") if f.strip() not in ("fp64", "fp32")]
        if bad or not (args.no_phonon and args.no_adjoint):
            sys.exit("--config mid12 takes --forms fp64,fp32 (no 16-bit instance at 12 orbitals) with "
                     "--no-phonon --no-adjoint")
    if args.config == "direct5":
        # a shape without a matrix-core instance (one neighbour more than the
        # instances): the direct fp64 kernel on the vector ALUs
        from paper_1912_10024_amd.inputs import Dims

        CONFIGS = dict(CONFIGS, direct5=Dims(nkz=7, ne=64, nqz=7, nw=10, na=1024, nb=5, norb=10, g_slots=1))
        CONFIG_INDEX = dict(CONFIG_INDEX, direct5=CONFIG_INDEX["mid"])
        if args.forms.strip() != "fp64" or not (args.no_phonon and args.no_adjoint):
            sys.exit("--config direct5 takes --forms fp64 (the direct kernel is fp64 only) with "
                     "--no-phonon --no-adjoint")
    direct = args.config == "direct5"
    d = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    if args.only_adjoint:
        rec = adjoint_record(args, sse, dev)
        print(json.dumps({"metric": "adjoint time, all three gradients (mid workload)",
                          "value": rec["ms_all_gradients"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": rec["ms_all_gradients"], "higher_is_better": False,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": rec["workload"]}, "adjoint": rec}), flush=True)
        return
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    t_gen = time.perf_counter()
    inp = generate_device(d, CONFIG_INDEX[args.config], device=dev)
    G, D, dH, nbr = inp["G<"], inp["D<"], inp["dH"], inp["nbr"]
    sse.check_nbr(nbr, d.na)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    f_eff = flops.f_eff(d)
    if args.only_phonon:
        rec = phonon_record(args, sse, flops, d, G, dH, nbr, dev)
        print(json.dumps({"metric": "phonon SSE useful TFLOP/s (Pi, one component)", "value": rec["value"],
                          "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": rec["workload"], "nkz": d.nkz, "ne": d.ne, "nqz": d.nqz,
                                     "nw": d.nw, "na": d.na, "nb": d.nb, "norb": d.norb, "g_slots": d.g_slots},
                          "roofline": rec["roofline"], "phonon": rec}), flush=True)
        return
    cpu = None
    if not args.no_cpu:
        f_block = f_eff / (d.nkz * d.ne * d.na)
        cpu, cpu_pts, cpu_ref = cpu_baseline(d, G, D, dH, nbr, args.cpu_seconds, f_block)
    peaks = {"fp64": FP64_MFMA_PEAK, "fp32": FP32_MFMA_PEAK, "bf16x2": FP16_MFMA_PEAK, "fp16x2": FP16_MFMA_PEAK,
             "fp16": FP16_MFMA_PEAK, "fp16_unscaled": FP16_MFMA_PEAK}
    # fp64: the useful flops of the regrouped form (GEMM and all twelve products
    # that form P; vector ALUs and matrix cores share the fp64 peak); fp32: the
    # fp32 matrix-core work (GEMM and the nine right products); 16-bit forms: the
    # four hi/lo partial products of both on the 16-bit matrix cores
    mfma_flops = {"fp64": flops.pd_useful_flops(d), "fp32": flops.pd_mfma_flops(d),
                  "bf16x2": flops.split16_mfma_flops(d), "fp16x2": flops.split16_mfma_flops(d),
                  "fp16": flops.single16_mfma_flops(d), "fp16_unscaled": flops.single16_mfma_flops(d)}
    whats = {"fp64": "useful fp64 flops: P.D GEMM + the 12 products forming P (X on the vector ALUs, X.gradH^H on "
                     "the matrix cores; one shared fp64 peak)",
             "fp32": "fp32 matrix-core flops: P.D GEMM + P = X.gradH^H products",
             "bf16x2": "16-bit matrix-core flops: 4 hi/lo products of the P.D GEMM and of P = X.gradH^H",
             "fp16x2": "16-bit matrix-core flops: 4 hi/lo products of the P.D GEMM and of P = X.gradH^H",
             "fp16": "16-bit matrix-core flops of the single-term form run on the split kernel: 2x the P.D GEMM, "
                     "4x P = X.gradH^H (flops.single16_mfma_flops)",
             "fp16_unscaled": "as fp16 (flops.single16_mfma_flops)"}
    traffic_records = {"fp64": ("fwd_mfma_device_traffic.txt", FWD_SOURCES),
                       "fp16x2": ("fwd_h16_device_traffic.txt", H16_SOURCES)}
    res = {}
    for form in forms:
        S = torch.empty(d.sigma_shape, dtype=torch.complex128, device=dev)
        ws = sse.workspace(d, form, device=dev)
        wall, kern_ms = time_form(sse, G, D, dH, nbr, S, ws, form, args.steps, args.warmup, dev)
        ms = float(np.mean(kern_ms))
        achieved = mfma_flops[form] / (ms * 1e-3)
        res[form] = {
            "value": f_eff / (ms * 1e-3) / 1e12,
            "ms_per_step": wall * 1e3 / args.steps,
            "kernel_ms": ms,
            "kernel_ms_all": [round(x, 3) for x in kern_ms],
            "roofline": {"bound": "mfma", "achieved": round(achieved / 1e12, 3), "peak": peaks[form] / 1e12,
                         "unit": "TFLOP/s", "frac": round(achieved / peaks[form], 4),
                         "traffic": (recorded_traffic(*traffic_records[form])
                                     if form in traffic_records and args.config == "device" else None),
                         "flops_per_launch": mfma_flops[form], "what": whats[form]},
        }
        if direct:
            # one dispatch of the direct kernel; its fp64 arithmetic runs on the
            # vector ALUs, whose fp64 peak equals the matrix cores' one
            res[form]["roofline"].update(bound="alu", dispatches_per_call=1,
                                         what="useful fp64 flops of the regrouped count (flops.pd_useful_flops), "
                                              "executed by the direct kernel on the vector ALUs")
        elif form in ("fp64", "fp32"):
            # this kernel runs as several dispatches per call; the roofline's launch
            # is the call (flops, traffic and HIP-event time all per call)
            res[form]["roofline"]["dispatches_per_call"] = fwd_mfma_dispatches(d, dev)
        if cpu is not None:
            res[form]["err"] = sampled_error(S, cpu_pts, cpu_ref)
        del S, ws
        torch.cuda.empty_cache()
    head = forms[0]
    line = {
        "metric": "SSE effective TFLOP/s (paper's regrouped flop count, one Sigma component), fp64 vs mixed",
        "value": round(res[head]["value"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[head]["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else head,
        "data": "synthetic",
        "config": {"workload": f"electron-phonon SSE Sigma^< forward ({args.config})",
                   "nkz": d.nkz, "ne": d.ne, "nqz": d.nqz, "nw": d.nw, "na": d.na, "nb": d.nb,
                   "norb": d.norb, "g_slots": d.g_slots},
        "kernel_ms": round(res[head]["kernel_ms"], 3),
        "f_eff": f_eff,
        "roofline": res[head]["roofline"],
        "executed_flops_per_launch": flops.pd_executed_flops(d),
        "input_gen_s": round(t_gen, 2),
        "forms": {f: {"value": round(r["value"], 3), "kernel_ms": round(r["kernel_ms"], 3),
                      "kernel_ms_all": r["kernel_ms_all"], "mfma_frac": r["roofline"]["frac"],
                      "speedup_vs_" + head: round(res[head]["kernel_ms"] / r["kernel_ms"], 3)}
                  for f, r in res.items()},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
        for f, r in res.items():
            line["forms"][f]["rel_err_vs_oracle_sampled"] = r["err"]
    if not args.no_phonon:
        line["phonon"] = phonon_record(args, sse, flops, d, G, dH, nbr, dev)
    if not args.no_adjoint:
        del G, D, dH, nbr, inp
        torch.cuda.empty_cache()
        line["adjoint"] = adjoint_record(args, sse, dev)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
