"""Throughput of the periodic background-charge FMM on one MI355X.

Default (the headline): one step = one fmm_energy_forces call (all of stages
a1-a13: sort, P2M, M2M, lattice operator, M2L, L2L, L2P, P2P, correction
terms, compensated energy reduction, forces scattered to the caller's order,
energy on the host) on the 1,000,000-atom box (333,333 rigid waters + one -1
ion, b = 215.30 A, levels 5, p = 12) with inputs resident in HBM.  Metric:
atom-evals/s = N * steps / time in mixed precision (FP32 P2P and M2L at the
fine levels; FP64 top levels, lattice, corrections and reduction); the FP64
FMM on the same box is timed beside it, and the oracle on a bounded sample on
the host cores.  Prints ONE JSON line.

Other workloads (each one JSON line):
  --config C5 [--p P] [--prec fp64|mixed|bf16|split16]   3,000,008 atoms, levels 6
  --config C5 --sweep       p in (4, 8, 12, 16) x (fp64, mixed, bf16, split16), one line each
  --config C4               32 charging windows (6k-48k atoms), one graph launch
                            of energies + forces and one of solute-solvent
                            energies per step, depths and P2P groups autotuned
                            (--autotune-cache FILE: taken from / stored in FILE)
--gpus > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M2L_IL = 875  # interaction-list size per cell
# dense MFMA peaks of MI355X (FP32, BF16, FP64, FP16) by precision mode
PEAK_TFLOPS = {"mixed": 157.3, "bf16": 2500.0, "fp64": 78.6, "split16": 2500.0}
PREC_NAMES = {"fp64": 0, "mixed": 1, "bf16": 2, "split16": 3}
DTYPES = {"mixed": "f32+f64", "fp64": "f64", "bf16": "bf16-m2l+f32+f64", "split16": "f16x3-m2l+f32+f64"}


def leaf_kernel(prec_name, info):
    """Name of the finest-level M2L kernel; info = fmm_plan_info of the plan.
    The FP32/FP64 kernel takes the symmetry-folded list (pairs or orbits of
    reflected offsets) in info["m2l_launches"] launches (row-class groups), the
    split-FP16 one the orbit list at p = 11, 12 and the plain list otherwise."""
    if prec_name == "bf16":
        return "k_m2l_bf16<false>"
    kind = {2: "orbit", 1: "pair", 0: "plain"}[info["m2l_scheme"]]
    if prec_name == "split16" and kind == "plain":
        return f"k_m2l_f16rows<false> x{info['m2l_launches']} (plain list, {info['m2l_entries']} entries)"
    t = {"fp64": "double", "split16": "PolF16x3F"}.get(prec_name, "float")
    return f"k_m2l_lds<{t}, false> x{info['m2l_launches']} ({kind} list, {info['m2l_entries']} entries)"


def m2l_entries(prec_name, info):
    return info["m2l_entries"]


def m2l_flops(p, level, entries):
    """Algorithmic M2L flops of one level: 2 K^2 per (target, list entry), an
    entry being one operator product (an offset for the BF16 kernel, a folded
    pair or orbit of offsets for the FP32/FP64 kernel)."""
    K = (p + 1) ** 2
    return 2.0 * K * K * entries * 8 ** level


def recorded_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "m2l_leaf_c3_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source sha256 of k_m2l\.hip: ([0-9a-f]{64})", text)
    m_b = re.search(r"HBM bytes per launch \(calibrated\): ([0-9.eE+]+)", text)
    m_k = re.search(r"kernel: (.+)", text)
    m_w = re.search(r"workload: (.+)", text)
    if not (m_src and m_b and m_k and m_w) or m_k.group(1).strip() != kernel or m_w.group(1).strip() != workload:
        return None
    src = os.path.join(ROOT, "paper_2003_13218_amd", "csrc", "k_m2l.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_src.group(1):
        return None
    return float(m_b.group(1))


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# sub-boxes of the benchmark's workload (waters at its density, one ion of
# its charge at the centre) that the oracle evaluates in full for the CPU
# baseline: about 64,000 and 256,000 atoms
CPU_SUBBOX_WATERS = (21333, 85333)


def _oracle_rate(w, accuracy):
    """Full-box oracle time extrapolated from two smaller boxes of the same workload.

    The oracle evaluates every atom of two seeded water boxes at the benchmark
    box's density (with its ion), each with its own balanced Ewald parameters
    for the truncation (the real-space cutoff that balances real and
    reciprocal work grows as N^(1/6), so the cost grows as N^(3/2)); the
    exponent fitted to the two timings carries the time to the benchmark's N."""
    import oracle
    import workloads
    z = float(w.q[w.mask.astype(bool)][0]) if w.mask.any() else 0.0
    sizes, times, params = [], [], []
    for k, nw in enumerate(CPU_SUBBOX_WATERS):
        b = workloads.box_for(nw)
        pos, q, _ = workloads.water_box(nw, b, [[b / 2] * 3], [z], 700 + k)
        kappa, rcut, kmax = oracle.ewald_params(b, accuracy, None, q.shape[0])
        t0 = time.perf_counter()
        oracle.ewald(pos, q, b, kappa=kappa, rcut=rcut, kmax=kmax)
        times.append(time.perf_counter() - t0)
        sizes.append(int(q.shape[0]))
        params.append({"atoms": sizes[-1], "box": round(b, 2), "kappa": round(kappa, 4), "rcut": round(rcut, 2),
                       "kmax": round(kmax, 3), "s": round(times[-1], 2)})
    alpha = math.log(times[1] / times[0]) / math.log(sizes[1] / sizes[0])
    t_full = times[1] * (w.n / sizes[1]) ** alpha
    return {"value": w.n / t_full, "t_full_s": round(t_full, 1), "accuracy": accuracy, "exponent": round(alpha, 3),
            "boxes": params}


def cpu_baseline(w, reference=False):
    """The oracle (as it stands) on the host cores with its balanced Ewald
    parameters at the truncation matched to the mixed-precision FMM's accuracy
    (1e-6, the value reported); with reference=True also at reference accuracy
    (1e-12).  Timed on two smaller boxes of the same workload and extrapolated
    to the benchmark's N (``_oracle_rate``)."""
    import oracle
    print(f"[bench] oracle at truncation 1e-6 on boxes of {CPU_SUBBOX_WATERS} waters ...", file=sys.stderr,
          flush=True)
    matched = _oracle_rate(w, 1e-6)
    print(f"[bench] ... {[b['s'] for b in matched['boxes']]} s", file=sys.stderr, flush=True)
    ref = None
    if reference:
        print("[bench] oracle at truncation 1e-12 ...", file=sys.stderr, flush=True)
        ref = _oracle_rate(w, 1e-12)
        print(f"[bench] ... {[b['s'] for b in ref['boxes']]} s", file=sys.stderr, flush=True)
    b0, b1 = matched["boxes"]
    return {"value": matched["value"], "unit": "atom-evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"FP64 Ewald (the oracle, every atom, energy + forces) with its balanced parameters at "
                       f"truncation 1e-6 on two seeded boxes of the same workload (waters at the benchmark's "
                       f"density plus its ion): {b0['atoms']} atoms in {b0['s']} s and {b1['atoms']} atoms in "
                       f"{b1['s']} s; time extrapolated to {w.n} atoms as t ~ N^{matched['exponent']} (fitted): "
                       f"{matched['t_full_s']} s"),
            "matched_accuracy": matched, "reference_accuracy": ref}


def sample_error(name, f, ph):
    """RMS relative force / potential error on the stored oracle sample."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_sample_oracle.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    idx = ref["idx"]
    fs, ps = f.cpu().numpy()[idx], ph.cpu().numpy()[idx]
    rel = lambda a, b: float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))  # noqa: E731
    return {"force_rms_rel": rel(fs, ref["force"]), "phi_rms_rel": rel(ps, ref["phi"]), "atoms": int(idx.size)}


def run_single(args, w, p, prec_name, steps, warmup, fp64_leg, cpu_leg, graph_leg=False):
    import torch
    import paper_2003_13218_amd as F
    pos = torch.tensor(w.pos, device="cuda")
    q = torch.tensor(w.q, device="cuda")
    plan = F.fmm_plan(w.box, w.levels, p)

    per_call = []

    def timed(prec, steps, warmup):
        F.fmm_plan_config(plan, prec)
        for _ in range(warmup):
            F.fmm_energy_forces(plan, pos, q)
        F.fmm_profile(plan, True)
        torch.cuda.synchronize()
        per_call.clear()
        t0 = time.perf_counter()
        e = None
        for _ in range(steps):
            # each call returns after its energy is on the host: the time
            # between returns is one whole evaluation
            t1 = time.perf_counter()
            e, _, _ = F.fmm_energy_forces(plan, pos, q)
            per_call.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stages, calls = F.fmm_profile_read(plan)
        F.fmm_profile(plan, False)
        return dt, e, {k: v / max(calls, 1) for k, v in stages.items()}

    prec = PREC_NAMES[prec_name]
    dt, e_main, st = timed(prec, steps, warmup)
    ms = 1e3 * dt / steps
    ms_median = 1e3 * sorted(per_call)[len(per_call) // 2]
    value = w.n * steps / dt
    print(f"[bench] {w.name} p={p} {prec_name}: {ms:.3f} ms/step, E = {e_main:.10f}", file=sys.stderr, flush=True)
    _, f, ph = F.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
    err = sample_error(w.name, f, ph)

    # dominant kernel: M2L at the finest level; algorithmic flops per launch
    # divided by its event-timed average duration on the plan's stream
    info = F.fmm_plan_info(plan)
    entries = m2l_entries(prec_name, info)
    flops_leaf = m2l_flops(p, w.levels, entries)
    m2l_ms = st["m2l_leaf"]
    achieved = flops_leaf / (m2l_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec_name]
    kernel = leaf_kernel(prec_name, info)
    workload = f"{w.name} levels {w.levels} p {p}"
    # Three counts of the same launch's work: the folded list it executes
    # (one K x K product per orbit of reflected offsets: achieved / frac), the
    # dense 875-offset list it is equivalent to (O_st = D_s O_t D_s, the
    # reflected operators differ by signs only), and what the matrix cores
    # issue including the class padding of the rows and the column padding.
    K = (p + 1) ** 2
    dense = m2l_flops(p, w.levels, M2L_IL)
    rows = info["m2l_rows"]
    cols = 32 * ((K + 31) // 32) if prec_name in ("bf16", "split16") else info["Kp"]
    # split operands: three FP16 products per operand pair
    executed = flops_leaf * (rows * cols) / (K * K) * (3 if prec_name == "split16" else 1)
    tflops = lambda f: f / (m2l_ms * 1e-3) / 1e12  # noqa: E731
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": recorded_traffic(kernel, workload),
                "kernel": f"{kernel} (M2L, level {w.levels})", "avg_ms": round(m2l_ms, 4),
                "flops_per_level": flops_leaf,
                "list_entries_per_cell": entries,
                "flops_counts": {"folded": flops_leaf, "dense_875_equivalent": dense,
                                 "executed_with_padding": executed},
                "frac_dense_equivalent": round(tflops(dense) / peak, 4),
                "frac_executed_with_padding": round(tflops(executed) / peak, 4),
                "folding": "profiles/m2l_folding.md"}
    desc = {"C3": "333,333 waters + one -1 ion", "C5": "1,000,000 waters + 8 ions (net +3)"}.get(w.name, w.name)
    metric = ("atom-evals/s (energy+forces) at 1M atoms, mixed vs FP64 FMM, rel err <=1e-5" if w.name == "C3"
              else f"atom-evals/s (energy+forces) on {w.name} ({w.n} atoms)")
    out = {
        "metric": metric,
        "value": value, "unit": "atom-evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "ms_per_call_median": round(ms_median, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[prec_name], "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} atoms ({desc}), b = {w.box} A, levels {w.levels}, p {p}, "
                               f"{prec_name} precision",
                   "n_atoms": w.n, "box": w.box, "levels": w.levels, "p": p, "precision": prec_name,
                   "fp64_tree_levels": info["fp64_levels"], "p2p_groups": info["p2p_groups"] or "auto"},
        "stages_ms": {k: round(v, 4) for k, v in st.items()},
        "sample_error": err,
        "roofline": roofline,
    }
    if graph_leg:
        # the same evaluation replayed as a captured HIP graph: a batch plan of
        # this one box (fmm_energy_forces_batch captures on its first call and
        # replays after; a graph branch keeps its near field on its own stream)
        import numpy as np
        gplan = F.fmm_plan_batch([w.box], p, levels=[w.levels])
        F.fmm_plan_config(gplan, prec)
        off = np.array([0, w.n], np.int64)
        for _ in range(2):
            F.fmm_energy_forces_batch(gplan, off, pos, q)
        torch.cuda.synchronize()
        gt = []
        for _ in range(steps):
            t1 = time.perf_counter()
            eg, _ = F.fmm_energy_forces_batch(gplan, off, pos, q)
            gt.append(time.perf_counter() - t1)
        gmed = sorted(gt)[len(gt) // 2]
        out["graph_replay"] = {"ms_per_call_median": round(1e3 * gmed, 4), "value": w.n / gmed,
                               "energy_rel_diff": abs(eg[0] - e_main) / abs(e_main)}
        F.fmm_destroy(gplan)
        print(f"[bench] graph replay: {1e3 * gmed:.3f} ms/call", file=sys.stderr, flush=True)
    if fp64_leg and prec_name != "fp64":
        n64 = max(3, steps // 4)
        dt64, e64, st64 = timed(F.FMM_FP64, n64, 1)
        out["fp64"] = {"value": w.n * n64 / dt64, "ms_per_step": 1e3 * dt64 / n64,
                       "ms_per_call_median": round(1e3 * sorted(per_call)[len(per_call) // 2], 4),
                       "stages_ms": {k: round(v, 4) for k, v in st64.items()}, "energy": e64}
        out["mixed_vs_fp64"] = value / out["fp64"]["value"]
        out["energy_rel_diff_vs_fp64"] = abs(e_main - e64) / abs(e64)
        print(f"[bench] fp64: {out['fp64']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if cpu_leg:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, reference=args.cpu_reference)
    F.fmm_destroy(plan)
    return out


UV_SCHEMES = {"symmetric": 0, "sparse": 1}


def run_batch(args):
    """C4: 32 charging windows, energies + forces and e_uv per step."""
    import numpy as np
    import torch
    import paper_2003_13218_amd as F
    import workloads
    ws = workloads.batch_windows()
    off = np.zeros(len(ws) + 1, np.int64)
    off[1:] = np.cumsum([w.n for w in ws])
    pos = torch.tensor(np.concatenate([w.pos for w in ws]), device="cuda")
    q = torch.tensor(np.concatenate([w.q for w in ws]), device="cuda")
    mask = torch.tensor(np.concatenate([w.mask for w in ws]), device="cuda")
    p = args.p or 10
    plan = F.fmm_plan_batch([w.box for w in ws], p, natoms=[w.n for w in ws])
    F.fmm_plan_config(plan, PREC_NAMES[args.prec])
    uv_scheme = UV_SCHEMES[args.uv_scheme]
    F.fmm_plan_options(plan, F.FMM_BOUNDARY_CONDUCTING, uv_scheme)
    model_levels, _ = F.fmm_batch_levels(plan)
    t0 = time.perf_counter()
    cache_hit = None
    if args.autotune_cache:
        cache_hit, levels, groups = F.fmm_autotune_batch_cached(plan, off, pos, q, args.autotune_cache)
    else:
        levels, groups = F.fmm_autotune_batch(plan, off, pos, q)
    t_tune = time.perf_counter() - t0
    for _ in range(args.warmup):
        F.fmm_energy_forces_batch(plan, off, pos, q)
        F.fmm_solute_solvent_energy_batch(plan, mask)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, _ = F.fmm_energy_forces_batch(plan, off, pos, q)
        U = F.fmm_solute_solvent_energy_batch(plan, mask)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = int(off[-1])
    print(f"[bench] C4: {1e3 * dt / args.steps:.3f} ms/step over {len(ws)} windows, {n} atoms",
          file=sys.stderr, flush=True)
    # the two calls of a step timed on their own (outside the timed region)
    split = {}
    for name, fn in (("energy_forces", lambda: F.fmm_energy_forces_batch(plan, off, pos, q)),
                     ("solute_solvent", lambda: F.fmm_solute_solvent_energy_batch(plan, mask))):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        split[name] = round(1e3 * (time.perf_counter() - t1) / args.steps, 3)
    # the other solute-solvent scheme, timed the same way
    other = "symmetric" if args.uv_scheme == "sparse" else "sparse"
    F.fmm_plan_options(plan, F.FMM_BOUNDARY_CONDUCTING, UV_SCHEMES[other])
    U_other = F.fmm_solute_solvent_energy_batch(plan, mask)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        F.fmm_solute_solvent_energy_batch(plan, mask)
    torch.cuda.synchronize()
    split[f"solute_solvent_{other}"] = round(1e3 * (time.perf_counter() - t1) / args.steps, 3)
    print(f"[bench] C4 split (ms/call): {split}", file=sys.stderr, flush=True)
    return {
        "metric": "atom-evals/s (energy+forces+solute-solvent energy), 32 charging windows, one graph launch each",
        "value": n * args.steps / dt, "unit": "atom-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {"workload": f"C4: {len(ws)} windows, {n} atoms (6k-48k per box), p {p}, {args.prec} precision",
                   "n_atoms": n, "windows": len(ws), "p": p, "precision": args.prec, "uv_scheme": args.uv_scheme,
                   "model_levels": model_levels.tolist(), "tuned_levels": levels.tolist(),
                   "tuned_p2p_groups": groups.tolist(), "autotune_s": round(t_tune, 2),
                   "autotune_cache_hit": cache_hit},
        "split_ms": split,
        "energies": E.tolist(), "e_uv": U.tolist(), f"e_uv_{other}": U_other.tolist(),
        "roofline": None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C3", choices=["C3", "C5", "C4"])
    ap.add_argument("--p", type=int, default=0, help="expansion order (default: the workload's)")
    ap.add_argument("--prec", default="mixed", choices=list(PREC_NAMES))
    ap.add_argument("--sweep", action="store_true", help="C5: p x precision sweep")
    ap.add_argument("--uv-scheme", default="sparse", choices=list(UV_SCHEMES),
                    help="C4: far-field scheme of the solute-solvent energy")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--autotune-cache", default="",
                    help="C4: depths and P2P groups through this cache file (tuned and stored on a miss)")
    ap.add_argument("--cpu-reference", action="store_true",
                    help="also time the oracle at reference accuracy (1e-12; minutes)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 5 times (the reference "
                         "kernel that scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not part of "
              "this build", file=sys.stderr)
        sys.exit(2)

    if args.copy_bytes:
        import torch
        n = args.copy_bytes // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 5}), flush=True)
        return
    import workloads
    if args.config == "C4":
        print(json.dumps(run_batch(args)), flush=True)
        return
    w = workloads.config(args.config)
    if args.sweep:
        for p in (4, 8, 12, 16):
            for prec in ("fp64", "mixed", "bf16", "split16"):
                out = run_single(args, w, p, prec, args.steps, args.warmup, False, False)
                print(json.dumps(out), flush=True)
        return
    p = args.p or w.p
    cpu_leg = not args.no_cpu and args.config == "C3"
    print(json.dumps(run_single(args, w, p, args.prec, args.steps, args.warmup, not args.no_fp64, cpu_leg,
                                graph_leg=not args.no_graph)), flush=True)


if __name__ == "__main__":
    main()
