"""Benchmark of the COLATUS hot path on one MI355X.

One step = one kick-drift-kick step of the paper-scale LCDM run: N = 32^3
particles, a from 1/51 to 1 in 1000 steps uniform in ln a, eps = 0.05 d,
k^-2 displacement initial conditions (synthetic, seeded), FP32 pair
arithmetic on tile-relative coordinates with TwoSum accumulation and FP64
state.  Each step is one O(N^2) pair sweep plus the O(N) finalise/kick/drift
kernel (launched eagerly, or replayed from a captured graph on runs of 32
steps or more).  ``value`` is pair interactions per second of the timed
steps, N^2 per step: K steps take K + 1 sweeps (the run evaluates the force
at its start positions once), and the extra sweep is counted as time only.

The same JSON line also carries, each measured in this process:
  roofline      the pair sweep's FP32 VALU throughput (20 flops per pair)
                against the MI355X FP32 vector peak, its average launch
                duration timed with hipEvents on the launching stream
  variants      the FP64 path, the run with per-step diagnostics (fused
                potential, energies, Layzer-Irvine), forward + adjoint, the
                ragged 256-box ensemble, and the O(N) integrator's bandwidth
  cpu_baseline  the FP64 oracle on this host's cores, on a bounded sample
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G pair-interactions/s & % FP32 peak at N=32^3: mixed vs FP64, fwd vs fwd+adj"
FLOPS_PER_PAIR = 20          # forward pair (rsqrt counted as 1)
FLOPS_PER_PAIR_ADJ = 36      # adjoint pair per cotangent (equal-mass minimal count)
PEAK_FP32 = 157.3e12         # MI355X FP32 vector peak (packed)
PEAK_FP64 = 78.6e12          # MI355X FP64 vector peak
PEAK_HBM = 8.0e12            # bytes/s


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pair_sweep_lcdm32_pmc.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "pair_sweep_lcdm32_valu_pmc.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_1208_3444_amd", "csrc", "pair_sweep.hip")


def slot_layout(N, precision):
    """(slots per particle, bytes per slot, grouped) of the forward sweep the
    library runs for one box of N: the symmetric form writes one slot per
    part of R x threads particles (P parts), or ceil(P/2) + 1 in 2x2 groups
    of part pairs (4 targets per lane, 64 threads, grouping on); FP32 slots
    with FP32 pairs and parts of at most 256, else FP64."""
    from paper_1208_3444_amd import colatus
    R, tpb, slices, form = colatus.tile_config(N, precision)
    grouped = (form == 2 and R == 4 and tpb == 64 and
               colatus.get_option(colatus.OPT_PAIR_GROUP) == 1)
    slots = ((slices + 1) // 2 + 1 if slices > 1 else 1) if grouped else slices
    slot_bytes = 12.0 if form == 2 and precision != "fp64" and R * tpb <= 256 else 24.0
    return slots, slot_bytes, grouped


def sweep_kernel_name(N, precision):
    from paper_1208_3444_amd import colatus
    R, tpb, slices, form = colatus.tile_config(N, precision)
    acc = {"mixed_twosum": "TwoSum", "mixed_f64acc": "FP64", "fp32": "FP32"}.get(precision,
                                                                               "FP64")
    if form == 2:
        t = "double" if precision == "fp64" else "float"
        slots, slot_bytes, grouped = slot_layout(N, precision)
        slot = "FP32" if slot_bytes == 12.0 else "FP64"
        if grouped:
            return (f"pair_sweep_sym_grp_kernel<{t}> (2x2 groups of part pairs, four waves "
                    f"per workgroup; {slots} {slot} slots per particle, summed in {acc} by "
                    f"the integrator)")
        return (f"pair_sweep_sym_kernel<{t}, R={R}, {tpb // 64} wave(s)> ({slots} {slot} "
                f"slots per particle, summed in {acc} by the integrator)")
    return f"pair_sweep_kernel<{acc}, R={R}, {tpb} threads, form {form}>"


def pmc_traffic():
    """HBM bytes per pair-sweep launch from the committed counter summary.

    The summary records FETCH_SIZE and WRITE_SIZE per dispatch, the factors
    that scale them to bytes (from a plain device copy of known size in the
    same runs) and the SHA-256 of the kernel source the counters were taken
    on; if that source has changed since, the figure no longer applies and
    None is returned.
    """
    import hashlib
    import re
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    src_hash = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    t = re.search(r"traffic bytes per launch: ([0-9.eE+-]+)", text)
    if not m or not t or m.group(1) != src_hash:
        return None
    return float(t.group(1))


def pmc_hw_flops():
    """FP32 flops the sweep's instructions perform per launch (the counter
    SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes) from the committed instruction-mix
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(VALU_SUMMARY):
        return None
    text = open(VALU_SUMMARY).read()
    src_hash = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
    m = re.search(r"source sha256 \(pair_sweep.hip\): ([0-9a-f]{64})", text)
    f = re.search(r"hardware FP32 flops per launch: ([0-9.eE+-]+)", text)
    if not m or not f or m.group(1) != src_hash:
        return None
    return float(f.group(1))


def trace_integrator_us():
    """The integrator's mean duration per launch in the committed kernel trace
    of this workload (no HIP events around the launches), or None if the
    integrator's source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "pair_sweep_lcdm32_kernel_stats.md")
    src = os.path.join(ROOT, "paper_1208_3444_amd", "csrc", "integrator.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"integrator.hip sha256: ([0-9a-f]{64})", text)
    row = re.search(r"\| `integrate_kernel` \| \d+ \| ([0-9.]+) \|", text)
    if not m or not row or m.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return float(row.group(1))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=300)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--precision", default="mixed_twosum")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--no-ftle", action="store_true",
                   help="skip the 64-tracer FTLE (192 cotangents, 200 steps, about 13 s)")
    p.add_argument("--cpu-sample-steps", type=int, default=30)
    p.add_argument("--integrator-64-only", action="store_true",
                   help="run only the integrator measurement at 64^3 (5 launches per precision) and print it as one JSON object, for counter runs")
    p.add_argument("--periodic-only", action="store_true",
                   help="run only the periodic-boundary measurement at 32^3 and print it as one "
                        "JSON object, for profiler runs")
    p.add_argument("--roctx", action="store_true",
                   help="roctx ranges around every library call (rocprofv3 --marker-trace)")
    p.add_argument("--calibration-copy-mib", type=int, default=0,
                   help="first run one plain elementwise pass over this many MiB (read "
                        "and write; a known-size kernel for scaling hardware byte counters)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1208_3444_amd import colatus, inputs
    if args.roctx:
        colatus.set_option(colatus.OPT_ROCTX, 1)

    dev = torch.device("cuda", 0)
    if args.calibration_copy_mib > 0:
        # one elementwise kernel that reads and writes exactly this many bytes
        # (torch's negation kernel, easy to pick out of a counter listing)
        n = args.calibration_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.integrator_64_only:
        ws3 = inputs.precision_sweep(64)
        x3, m3 = torch.from_numpy(ws3.x).to(dev), torch.from_numpy(ws3.m).to(dev)
        print(json.dumps({"integrator_64cubed": integrator_64cubed(ws3, x3, m3, colatus, torch)}), flush=True)
        return
    w = inputs.lcdm_grf(32)
    H_i = colatus.hubble(w.a_begin, w.cosmo)
    v0 = w.velocities(H_i)
    N = w.N
    pairs = float(N) * N
    if args.periodic_only:
        print(json.dumps({"periodic_32cubed": periodic_32cubed(w, v0, args, colatus, np, torch,
                                                               dev)}), flush=True)
        return

    def state():
        return (torch.from_numpy(w.x.copy()).to(dev), torch.from_numpy(v0.copy()).to(dev),
                torch.from_numpy(w.m.copy()).to(dev))

    K, W = args.steps, args.warmup
    if W + K > w.n_steps:
        raise SystemExit(f"--warmup + --steps must be <= {w.n_steps}")

    def timed_run(x, v, m, first, last, prec, diag=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
                    first_step=first, last_step=last, precision=prec, diag=diag)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # ---- roofline: pair-sweep launches timed with hipEvents ---------------
    # Measured first, on a copy of the start state: 100 untimed steps that
    # bring the GPU to its steady clock, then 200 eagerly launched steps with
    # each sweep and integrator launch bracketed by hipEvents on the
    # launching stream.  (The GPU is therefore warm before the headline's own
    # warm-up steps as well.)
    R_WARM, R_STEPS = 100, 200
    xr_, vr_, mr_ = state()
    timed_run(xr_, vr_, mr_, 0, R_WARM, args.precision)
    colatus.set_option(colatus.OPT_TIMER, 1)
    colatus.timer_read(0, reset=True)
    colatus.timer_read(2, reset=True)
    timed_run(xr_, vr_, mr_, R_WARM, R_WARM + R_STEPS, args.precision)
    ms_tot, launches = colatus.timer_read(0, reset=True)
    int_ms, int_launches = colatus.timer_read(2, reset=True)
    colatus.set_option(colatus.OPT_TIMER, 0)
    del xr_, vr_, mr_
    sweep_ms = ms_tot / launches
    achieved = FLOPS_PER_PAIR * pairs / (sweep_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": pmc_traffic(),
                "kernel": sweep_kernel_name(N, args.precision), "launch_ms": sweep_ms,
                "launches": launches,
                "flops_per_launch": FLOPS_PER_PAIR * pairs,
                "note": "algorithmic: 20 flops per ordered pair, N^2 ordered pairs per "
                        "launch; the symmetric loop evaluates each unordered pair once "
                        "and applies it to both particles (hw_frac: the FP32 flops its "
                        "instructions perform, from the counters); measured over steps "
                        f"{R_WARM}-{R_WARM + R_STEPS} of the run, before the headline"}
    hw = pmc_hw_flops()
    roofline["hw_flops_per_launch"] = hw
    roofline["hw_frac"] = None if hw is None else hw / (sweep_ms * 1e-3) / PEAK_FP32
    print(f"[bench] pair sweep {sweep_ms:.4f} ms/launch -> {achieved / 1e12:.2f} TFLOP/s",
          file=sys.stderr, flush=True)

    # ---- headline: mixed forward run steps -------------------------------
    x, v, m = state()
    timed_run(x, v, m, 0, W, args.precision)
    print(f"[bench] warmup {W} steps done", file=sys.stderr, flush=True)
    t = timed_run(x, v, m, W, W + K, args.precision)
    value = K * pairs / t / 1e9
    ms_per_step = 1e3 * t / K
    print(f"[bench] timed {K} steps: {ms_per_step:.3f} ms/step, {value:.1f} Gpairs/s",
          file=sys.stderr, flush=True)

    # the O(N) integrator (finalise the slice partials, kick, drift): HBM-
    # bound; algorithmic bytes per particle = read S partial-sum slots (3
    # components, FP32 or FP64), x and p (48 B); write x and p (48 B)
    slices, slot_bytes, _ = slot_layout(N, args.precision)
    int_bytes = N * (slot_bytes * slices + 96.0)
    int_launch_ms = int_ms / int_launches
    trace_us = trace_integrator_us()
    integrator = {"bound": "hbm", "launch_us": 1e3 * int_launch_ms,
                  "bytes_per_launch": int_bytes,
                  "achieved_GBs": int_bytes / (int_launch_ms * 1e-3) / 1e9,
                  "peak_GBs": PEAK_HBM / 1e9,
                  "frac": int_bytes / (int_launch_ms * 1e-3) / PEAK_HBM,
                  "trace_us": trace_us,
                  "frac_trace": None if trace_us is None else
                  int_bytes / (trace_us * 1e-6) / PEAK_HBM,
                  "note": f"{slices} partial-sum slots per particle, {slot_bytes:.0f} B each "
                          f"({slot_bytes * slices * N / 1e6:.0f} MB at this N); launch_us is "
                          "timed with HIP events around each launch, which add a few us to a "
                          "launch this short; trace_us is the mean of the committed kernel "
                          "trace of this workload (no events), used while the integrator's "
                          "source is unchanged"}

    line = {
        "metric": METRIC, "value": value, "unit": "Gpairs/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_per_step, "steps_per_s": 1e3 / ms_per_step,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "lcdm_grf_32^3", "N": N, "cosmology": "LCDM Om_M=0.3 Om_L=0.7",
                   "a_begin": w.a_begin, "a_end": w.a_end, "n_steps_grid": w.n_steps,
                   "eps": w.eps, "precision": args.precision,
                   "pairs_per_step": pairs, "sweeps_timed": K + 1,
                   "pairs_counted": "N^2 per step (the start-of-call sweep is not counted)",
                   "seed": w.seed},
        "roofline": roofline,
        "integrator": integrator,
    }

    if not args.no_variants:
        line["variants"] = variants(w, v0, state, timed_run, args, colatus, inputs, np, torch,
                                    dev)
        # mixed / FP64 throughput: the forward (headline against the FP64 call) and the
        # forward + adjoint
        var = line["variants"]
        if args.precision != "fp64":
            var["fp64_fwd"]["mixed_over_fp64"] = value / var["fp64_fwd"]["gpairs_s"]
            var["fp64_fwd_adj"]["mixed_over_fp64"] = (var["mixed_fwd_adj"]["gpairs_s"]
                                                      / var["fp64_fwd_adj"]["gpairs_s"])

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, v0, args)

    print(json.dumps(line), flush=True)


def variants(w, v0, state, timed_run, args, colatus, inputs, np, torch, dev):
    out = {}
    N = w.N
    pairs = float(N) * N
    # FP64 path, same workload
    x, v, m = state()
    Kd = 200  # like the headline, a long call: its start-of-call sweep is 0.5 %
    timed_run(x, v, m, 0, 5, "fp64")
    t = timed_run(x, v, m, 5, 5 + Kd, "fp64")
    colatus.set_option(colatus.OPT_TIMER, 1)
    colatus.timer_read(0, reset=True)
    timed_run(x, v, m, 5 + Kd, 5 + 2 * Kd, "fp64")
    ms_tot, launches = colatus.timer_read(0, reset=True)
    colatus.set_option(colatus.OPT_TIMER, 0)
    fp64_rate = Kd * pairs / t / 1e9
    out["fp64_fwd"] = {"gpairs_s": fp64_rate, "ms_per_step": 1e3 * t / Kd,
                       "sweep_ms": ms_tot / launches,
                       "frac_fp64_peak": FLOPS_PER_PAIR * pairs / (ms_tot / launches * 1e-3)
                       / PEAK_FP64}
    print(f"[bench] fp64: {fp64_rate:.1f} Gpairs/s", file=sys.stderr, flush=True)

    # the paper-scale run in full, 1000 steps from a = 1/51 to 1, in FP64 and
    # mixed, each with per-step diagnostics (one call each, timed), and the
    # chaos control of the Layzer-Irvine comparison: the FP64 run started
    # from positions perturbed at the FP32 rounding level, x (1 + 2^-24 u)
    u = np.random.default_rng(11).choice([-1.0, 1.0], size=w.x.shape)
    full = {}
    for key, prec, x0 in (("fp64", "fp64", w.x), (args.precision, args.precision, w.x),
                          ("fp64_control", "fp64", w.x * (1 + 2.0 ** -24 * u))):
        x = torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
        v = torch.from_numpy(v0.copy()).to(dev)
        m = torch.from_numpy(w.m.copy()).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
                        precision=prec, diag=True)
        torch.cuda.synchronize()
        full[key] = (time.perf_counter() - t0, d)
    ref = full["fp64"][1]
    scale = float(np.abs(ref["U"]).max())

    def departure(d, thr):
        idx = np.nonzero(np.abs(d["LI"] - ref["LI"]) / scale > thr)[0]
        return float(ref["a"][idx[0]]) if len(idx) else None

    run1000 = {}
    for key, (t, d) in full.items():
        run1000[key] = {"seconds": t, "ms_per_step": 1e3 * t / w.n_steps,
                        "gpairs_s": w.n_steps * pairs / t / 1e9,
                        "LI_end_over_maxU": float(d["LI"][-1] / scale),
                        "LI_max_over_maxU": float(np.abs(d["LI"]).max() / scale)}
        if key != "fp64":
            run1000[key]["max_dLI_vs_fp64_over_maxU"] = float(
                np.abs(d["LI"] - ref["LI"]).max() / scale)
            run1000[key]["a_where_dLI_exceeds"] = {f"{thr:g}": departure(d, thr)
                                                   for thr in (1e-8, 1e-6, 1e-4)}
    out["lcdm32_1000_steps_with_diagnostics"] = run1000
    print(f"[bench] 1000-step runs: fp64 {run1000['fp64']['seconds']:.3f} s, "
          f"{args.precision} {run1000[args.precision]['seconds']:.3f} s; LI end/max|U| "
          f"{run1000['fp64']['LI_end_over_maxU']:.4f} / "
          f"{run1000[args.precision]['LI_end_over_maxU']:.4f}", file=sys.stderr, flush=True)

    # the EdS 16^3 lattice run in full: 64 steps from a = 0.1 to 1, FP64 and
    # mixed (4096 particles: the small-box tile shape; a whole call is about
    # a millisecond, so one untimed call, then the best of three)
    we = inputs.eds_lattice(16)
    ve0 = we.velocities(colatus.hubble(we.a_begin, we.cosmo))
    eds = {}
    for prec in ("fp64", args.precision):
        times = []
        for rep in range(4):
            xe_, ve_, me_ = (torch.from_numpy(a.copy()).to(dev) for a in (we.x, ve0, we.m))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            colatus.run(xe_, ve_, me_, we.eps, we.G, we.cosmo, we.a_begin, we.a_end, we.n_steps,
                        precision=prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = min(times[1:])
        eds[prec] = {"seconds_64_steps": t, "ms_per_step": 1e3 * t / we.n_steps,
                     "gpairs_s": we.n_steps * float(we.N) ** 2 / t / 1e9,
                     "tile": list(colatus.tile_config(we.N, prec))}
    out["eds_lattice_16cubed_64_steps"] = eds

    # mixed with per-step diagnostics (fused potential + energies + LI)
    x, v, m = state()
    Kg = 100
    timed_run(x, v, m, 0, 5, args.precision, diag=True)
    t = timed_run(x, v, m, 5, 5 + Kg, args.precision, diag=True)
    out["mixed_fwd_diag"] = {"gpairs_s": Kg * pairs / t / 1e9,
                             "ms_per_step": 1e3 * t / Kg}

    # the same run with the Eq. (10) deformation attractor at the box centre
    # (strength 0.05, a tenth of the box mass in units of G m): O(N) work
    x, v, m = state()
    att = (0.05, (0.5, 0.5, 0.5))
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=0,
                last_step=5, precision=args.precision, attractor=att)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=5,
                last_step=5 + Kg, precision=args.precision, attractor=att)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["mixed_fwd_attractor"] = {"gpairs_s": Kg * pairs / t / 1e9,
                                  "ms_per_step": 1e3 * t / Kg, "attractor": [0.05, 0.5, 0.5, 0.5]}

    # the same run with the Eq. (6) background term (b = Om_M H0^2 / 2 about the
    # box centre): O(N) work; the whole run's Layzer-Irvine residual, now
    # without the open box's collapse
    x, v, m = state()
    bg = (colatus.background_coefficient(w.cosmo), (0.5, 0.5, 0.5))
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=0,
                last_step=5, precision=args.precision, background=bg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=5,
                last_step=5 + Kg, precision=args.precision, background=bg)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    x, v, m = state()
    d = colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
                    precision=args.precision, diag=True, background=bg)
    u = np.abs(d["U"]).max()
    out["mixed_fwd_background"] = {"gpairs_s": Kg * pairs / t / 1e9,
                                   "ms_per_step": 1e3 * t / Kg, "b": bg[0],
                                   "LI_end_over_maxU_1000_steps": float(abs(d["LI"][-1]) / u)}

    # the paper's difference equations, Eqs. (3)-(5): throughput over the
    # timed steps, and the Layzer-Irvine residual of the whole 1000-step run
    # against the kick-drift-kick scheme's (the paper calls the former not
    # symplectic)
    x, v, m = state()
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=0,
                last_step=5, precision=args.precision, scheme="he")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=5,
                last_step=5 + Kg, precision=args.precision, scheme="he")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    li = {}
    for scheme in ("kdk", "he"):
        x, v, m = state()
        d = colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
                        precision=args.precision, diag=True, scheme=scheme)
        u = np.abs(d["U"]).max()
        li[scheme] = {"LI_end_over_maxU": float(abs(d["LI"][-1]) / u),
                      "LI_max_over_maxU": float(np.abs(d["LI"]).max() / u)}
    # one sweep per step (the force at the half step; none at the grid points)
    out["he_difference_equations"] = {"gpairs_s": Kg * pairs / t / 1e9,
                                      "ms_per_step": 1e3 * t / Kg,
                                      "layzer_irvine_1000_steps": li}
    print(f"[bench] Eqs. (3)-(5): {out['he_difference_equations']['gpairs_s']:.1f} Gpairs/s; "
          f"LI/U kdk {li['kdk']['LI_max_over_maxU']:.2e} he {li['he']['LI_max_over_maxU']:.2e}",
          file=sys.stderr, flush=True)

    # tracer tracks of 64 particles at every grid point over the timed steps,
    # then the velocity power spectrum of their whole 1000-step tracks
    # (timed back to back with the same steps untracked, from the same state)
    tr = np.random.default_rng(55).choice(N, 64, replace=False)
    tt = {}
    for key, trc in (("untracked", None), ("tracked", tr), ("untracked", None),
                     ("tracked", tr)):
        x, v, m = state()
        colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=0,
                    last_step=5, precision=args.precision, tracers=trc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps, first_step=5,
                    last_step=5 + Kg, precision=args.precision, tracers=trc)
        torch.cuda.synchronize()
        tt[key] = time.perf_counter() - t0  # the second of each pair is kept
    t = tt["tracked"]
    x, v, m = state()
    _, track = colatus.run(x, v, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
                           precision=args.precision, tracers=tr)
    colatus.velocity_spectrum(track, remove_mean=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(10):
        colatus.velocity_spectrum(track, remove_mean=True)
    torch.cuda.synchronize()
    out["tracks_64"] = {"gpairs_s": Kg * pairs / t / 1e9, "ms_per_step": 1e3 * t / Kg,
                        "untracked_ms_per_step": 1e3 * tt["untracked"] / Kg,
                        "track_rows": int(track.shape[0]),
                        "spectrum_ms": 1e3 * (time.perf_counter() - t1) / 10}
    print(f"[bench] 64 tracers: {out['tracks_64']['gpairs_s']:.1f} Gpairs/s; spectrum of "
          f"{track.shape[0]} rows {out['tracks_64']['spectrum_ms']:.3f} ms",
          file=sys.stderr, flush=True)

    # forward + adjoint (adjoint workload recipe, 200 steps from a = 0.2,
    # checkpoints every 20), one cotangent: the tracers' |v|^2 loss
    wa = inputs.adjoint_run(32)
    va = wa.velocities(colatus.hubble(wa.a_begin, wa.cosmo))
    xa, vat, ma = (torch.from_numpy(a.copy()).to(dev) for a in (wa.x, va, wa.m))
    lx = torch.zeros_like(xa)
    lv = torch.zeros_like(xa)
    tr = torch.from_numpy(wa.extra["tracers"]).to(dev)
    lv[:, tr] = 1.0
    nA = 40
    for prec in (args.precision, "fp64"):
        colatus.adjoint(xa, vat, ma, wa.eps, wa.G, wa.cosmo, wa.a_begin, wa.a_end, 4, lx, lv,
                        checkpoint_every=2, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colatus.adjoint(xa, vat, ma, wa.eps, wa.G, wa.cosmo, wa.a_begin, wa.a_end, nA, lx, lv,
                        checkpoint_every=wa.extra["checkpoint_every"], precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        fwd_sweeps = (nA + 1) + nA   # forward + recompute
        adj_sweeps = nA + 1
        flops = (FLOPS_PER_PAIR * fwd_sweeps + FLOPS_PER_PAIR_ADJ * adj_sweeps) * pairs
        peak = PEAK_FP64 if prec == "fp64" else PEAK_FP32
        key = "fp64_fwd_adj" if prec == "fp64" else "mixed_fwd_adj"
        out[key] = {"gpairs_s": (fwd_sweeps + adj_sweeps) * pairs / t / 1e9,
                    "ms_per_step": 1e3 * t / nA, "tflops": flops / t / 1e12,
                    "frac_peak": flops / t / peak, "steps": nA,
                    "flops_per_adjoint_pair": FLOPS_PER_PAIR_ADJ}
        print(f"[bench] {key}: {out[key]['gpairs_s']:.1f} Gpairs/s", file=sys.stderr,
              flush=True)

    # the full adjoint workload: 200 steps from a = 0.2, checkpoints every 20,
    # the tracers' summed squared final velocity (one cotangent)
    x4, v4, m4 = (torch.from_numpy(a.copy()).to(dev) for a in (wa.x, va, wa.m))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.adjoint(x4, v4, m4, wa.eps, wa.G, wa.cosmo, wa.a_begin, wa.a_end, wa.n_steps,
                    lx, lv, checkpoint_every=wa.extra["checkpoint_every"],
                    precision=args.precision)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    nS = wa.n_steps
    out["adjoint_200_steps"] = {
        "seconds": t, "forward_sweeps": 2 * nS + 1, "adjoint_sweeps": nS + 1,
        "gpairs_s": (3 * nS + 2) * pairs / t / 1e9,
        "tflops": (FLOPS_PER_PAIR * (2 * nS + 1) + FLOPS_PER_PAIR_ADJ * (nS + 1)) * pairs / t
        / 1e12}
    # the same run keeping every position (158 MB at 32^3) instead of
    # recomputing the segments: one force sweep per step fewer, same bits
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.adjoint(x4, v4, m4, wa.eps, wa.G, wa.cosmo, wa.a_begin, wa.a_end, wa.n_steps,
                    lx, lv, checkpoint_every=0, precision=args.precision)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["adjoint_200_steps_all_positions_kept"] = {
        "seconds": t, "forward_sweeps": nS + 1, "adjoint_sweeps": nS + 1,
        "gpairs_s": (2 * nS + 2) * pairs / t / 1e9,
        "tflops": (FLOPS_PER_PAIR * (nS + 1) + FLOPS_PER_PAIR_ADJ * (nS + 1)) * pairs / t / 1e12,
        "position_bytes": 24.0 * wa.N * (nS + 1)}
    if not args.no_ftle:
        tr = [int(i) for i in wa.extra["tracers"]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam_t, lam_lna, _ = colatus.ftle(x4, v4, m4, wa.eps, wa.G, wa.cosmo, wa.a_begin,
                                         wa.a_end, wa.n_steps, tr,
                                         checkpoint_every=wa.extra["checkpoint_every"],
                                         precision=args.precision)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        lam_lna = lam_lna.cpu().numpy()
        out["ftle_192_cotangents"] = {"seconds": t, "tracers": len(tr),
                                      "lambda_per_ln_a_median": float(np.median(lam_lna)),
                                      "lambda_per_ln_a_max": float(np.max(lam_lna))}
        print(f"[bench] FTLE of {len(tr)} tracers (192 cotangents): {t:.1f} s",
              file=sys.stderr, flush=True)
    print(f"[bench] adjoint 200 steps: {out['adjoint_200_steps']['seconds']:.3f} s "
          f"(every position kept: "
          f"{out['adjoint_200_steps_all_positions_kept']['seconds']:.3f} s)",
          file=sys.stderr, flush=True)

    per = periodic_32cubed(w, v0, args, colatus, np, torch, dev)
    out["periodic_32cubed"] = per

    # single force evaluation at N = 64^3 in each precision
    ws3 = inputs.precision_sweep(64)
    x3, m3 = torch.from_numpy(ws3.x).to(dev), torch.from_numpy(ws3.m).to(dev)
    pairs3 = float(ws3.N) ** 2
    sweep = {}
    for prec in ("fp32", "mixed_twosum", "mixed_f64acc", "fp64"):
        for _ in range(3):
            colatus.forces(x3, m3, ws3.eps, a=0.5, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            colatus.forces(x3, m3, ws3.eps, a=0.5, precision=prec)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / 10
        sweep[prec] = {"ms": 1e3 * t, "gpairs_s": pairs3 / t / 1e9}
    out["precision_sweep_64cubed"] = sweep

    integ = integrator_64cubed(ws3, x3, m3, colatus, torch)
    out["integrator_64cubed"] = integ
    print(f"[bench] integrator at 64^3: {integ['mixed_twosum']['achieved_GBs']:.0f} GB/s "
          f"(FP32 slots), {integ['fp64']['achieved_GBs']:.0f} GB/s (FP64)", file=sys.stderr,
          flush=True)

    # ragged ensemble: 256 boxes, N log-uniform in [512, 8192], one launch per step
    e = inputs.ragged_ensemble()
    ve = e.velocities(colatus.hubble(e.a_begin, e.cosmo))
    xe, vee, me = (torch.from_numpy(a.copy()).to(dev) for a in (e.x, ve, e.m))
    sizes = np.diff(e.box_offsets)
    pairs_e = float(np.sum(sizes.astype(np.float64) ** 2))
    batch = (e.box_offsets, e.box_eps)

    def erun(first, last):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colatus.run(xe, vee, me, 0.0, e.G, e.cosmo, e.a_begin, e.a_end, e.n_steps,
                    first_step=first, last_step=last, precision=args.precision, batch=batch)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # a warm-up run as long as the timed one (the first batched runs of a
    # process ran up to 15 % slower)
    Ke = 50
    erun(0, Ke)
    t = erun(Ke, 2 * Ke)
    ens = {"boxes": int(len(sizes)), "particles": int(sizes.sum()),
           "pairs_per_step": pairs_e, "gpairs_s": Ke * pairs_e / t / 1e9,
           "ms_per_step": 1e3 * t / Ke}
    # the per-box loop: each box its own run call (the plain kernels, no batching)
    xs = [(xe[:, o0:o1].contiguous(), vee[:, o0:o1].contiguous(), me[o0:o1].contiguous())
          for o0, o1 in zip(e.box_offsets[:-1], e.box_offsets[1:])]
    Kl = 5
    # an untimed pass first builds each box's work list (the library keeps
    # them), so the timed loop measures the per-box calls themselves
    for b, (xb, vb, mb) in enumerate(xs):
        colatus.run(xb, vb, mb, float(e.box_eps[b]), e.G, e.cosmo, e.a_begin, e.a_end,
                    e.n_steps, first_step=2 * Ke - 1, last_step=2 * Ke,
                    precision=args.precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, (xb, vb, mb) in enumerate(xs):
        colatus.run(xb, vb, mb, float(e.box_eps[b]), e.G, e.cosmo, e.a_begin, e.a_end,
                    e.n_steps, first_step=2 * Ke, last_step=2 * Ke + Kl,
                    precision=args.precision)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ens["per_box_loop_gpairs_s"] = Kl * pairs_e / t / 1e9
    ens["speedup_vs_per_box_loop"] = ens["gpairs_s"] / ens["per_box_loop_gpairs_s"]
    # the same batched step with the persistent grid (work items pulled from a
    # device counter), and with tile shapes from the autotuner
    colatus.set_option(colatus.OPT_PERSISTENT, 1)
    erun(2 * Ke, 2 * Ke + 5)
    t = erun(2 * Ke + 5, 3 * Ke + 5)
    colatus.set_option(colatus.OPT_PERSISTENT, 0)
    ens["persistent_grid_gpairs_s"] = Ke * pairs_e / t / 1e9
    colatus.set_option(colatus.OPT_AUTOTUNE, 1)
    erun(3 * Ke + 5, 3 * Ke + 10)
    t = erun(3 * Ke + 10, 4 * Ke + 10)
    colatus.set_option(colatus.OPT_AUTOTUNE, 0)
    ens["autotuned_gpairs_s"] = Ke * pairs_e / t / 1e9
    out["ensemble_256"] = ens
    print(f"[bench] ensemble: {ens['gpairs_s']:.1f} Gpairs/s "
          f"({ens['speedup_vs_per_box_loop']:.1f}x per-box loop)", file=sys.stderr, flush=True)
    return out


def periodic_32cubed(w, v0, args, colatus, np, torch, dev):
    """Periodic boundaries (Ewald summation) on the 32^3 positions in a unit
    box: one force evaluation per precision (real-space pair sweep and
    reciprocal-space sums), and 20 steps of the periodic run."""
    per = {}
    xp, mp = (torch.from_numpy(a.copy()).to(dev) for a in (w.x, w.m))
    for prec in ("fp64", args.precision):
        for _ in range(2):
            colatus.forces_periodic(xp, mp, w.eps, 1.0, a=w.a_begin, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            colatus.forces_periodic(xp, mp, w.eps, 1.0, a=w.a_begin, precision=prec)
        torch.cuda.synchronize()
        per[prec] = {"force_ms": 1e3 * (time.perf_counter() - t0) / 5}
    xr_, vr_ = (torch.from_numpy(a.copy()).to(dev) for a in (w.x, v0))
    colatus.run_periodic(xr_, vr_, mp, w.eps, w.G, w.cosmo, 1.0, w.a_begin, w.a_end, w.n_steps,
                         first_step=0, last_step=5, precision=args.precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colatus.run_periodic(xr_, vr_, mp, w.eps, w.G, w.cosmo, 1.0, w.a_begin, w.a_end, w.n_steps,
                         first_step=5, last_step=25, precision=args.precision)
    torch.cuda.synchronize()
    per[args.precision]["run_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / 20
    print(f"[bench] periodic 32^3: force fp64 {per['fp64']['force_ms']:.3f} ms, "
          f"{args.precision} {per[args.precision]['force_ms']:.3f} ms; run "
          f"{per[args.precision]['run_ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    return per


def integrator_64cubed(ws3, x3, m3, colatus, torch):
    """The integrator beyond the 256 MB Infinity Cache: at 64^3 its 513 slots
    per particle (1024 parts in 2x2 groups) are 1.6 GB (FP32 slots) or 3.2 GB
    (FP64 pairs) per launch.
    A 4-step run per precision, its integrator launches timed with hipEvents."""
    v3 = torch.zeros_like(x3)
    integ = {}
    for prec in ("mixed_twosum", "fp64"):
        xs3 = x3.clone()
        colatus.set_option(colatus.OPT_TIMER, 1)
        colatus.timer_read(2, reset=True)
        colatus.run(xs3, v3, m3, ws3.eps, ws3.G, ws3.cosmo, 0.5, 0.52, 4, precision=prec)
        torch.cuda.synchronize()
        ms, launches = colatus.timer_read(2, reset=True)
        colatus.set_option(colatus.OPT_TIMER, 0)
        s3, sb, _ = slot_layout(ws3.N, prec)
        nbytes = ws3.N * (sb * s3 + 96.0)
        integ[prec] = {"launch_ms": ms / launches, "bytes_per_launch": nbytes,
                       "achieved_GBs": nbytes / (ms / launches * 1e-3) / 1e9,
                       "frac_hbm_peak": nbytes / (ms / launches * 1e-3) / PEAK_HBM,
                       "slots": s3, "slot_bytes": sb, "launches": launches}
    return integ


def cpu_baseline(w, v0, args):
    import oracle
    n = args.cpu_sample_steps
    t0 = time.perf_counter()
    oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps,
               first_step=0, last_step=n)
    t = time.perf_counter() - t0
    sweeps = n + 1
    rate = sweeps * float(w.N) ** 2 / t / 1e9
    print(f"[bench] cpu oracle: {rate:.3f} Gpairs/s in {t:.1f} s", file=sys.stderr, flush=True)
    cores = oracle.num_threads()
    # single FP64 force evaluations (median of 3) at the three workload sizes,
    # and one 32^3 evaluation on a single core
    import statistics
    detail = {"cpu_model": _cpu_model(), "threads": cores}
    for name, ww, tg in (("eds_lattice_16^3", _inputs().eds_lattice(16), None),
                         ("lcdm_grf_32^3", w, None),
                         ("precision_sweep_64^3_4096_targets", _inputs().precision_sweep(64),
                          "targets")):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            if tg is None:
                oracle.forces(ww.x, ww.m, ww.eps, G=ww.G)
            else:
                oracle.forces_targets(ww.x, ww.m, ww.extra[tg], ww.eps, G=ww.G)
            ts.append(time.perf_counter() - t0)
        npairs = float(ww.N) * (ww.N if tg is None else len(ww.extra[tg]))
        detail[name] = {"seconds_median_of_3": statistics.median(ts),
                        "gpairs_s": npairs / statistics.median(ts) / 1e9}
    # ten steps of the 16^3 EdS lattice run (11 force sweeps)
    w1 = _inputs().eds_lattice(16)
    c1 = w1.cosmo
    v1 = w1.velocities(oracle.hubble(w1.a_begin, c1["H0"], c1["Om_R"], c1["Om_M"], c1["Om_K"],
                                     c1["Om_L"]))
    t0 = time.perf_counter()
    oracle.run(w1.x, v1, w1.m, w1.eps, w1.G, w1.cosmo, w1.a_begin, w1.a_end, w1.n_steps,
               first_step=0, last_step=10)
    t1 = time.perf_counter() - t0
    detail["eds_lattice_16^3_10_steps"] = {"seconds": t1,
                                           "gpairs_s": 11 * float(w1.N) ** 2 / t1 / 1e9}
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.forces(w.x, w.m, w.eps, G=w.G)
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    detail["lcdm_grf_32^3_one_core"] = {"seconds": t1, "gpairs_s": float(w.N) ** 2 / t1 / 1e9}
    print(f"[bench] cpu oracle, one core: {detail['lcdm_grf_32^3_one_core']['gpairs_s']:.3f} "
          f"Gpairs/s", file=sys.stderr, flush=True)
    return {"value": rate, "unit": "Gpairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} kick-drift-kick steps ({sweeps} FP64 force sweeps) of the "
                      f"same 32^3 LCDM run", "seconds": t, "detail": detail}


def _inputs():
    from paper_1208_3444_amd import inputs
    return inputs


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
