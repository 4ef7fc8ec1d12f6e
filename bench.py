"""Benchmark of the GM-HC-CN implicit step on one MI355X.

Workload (default): 2D mixed two-stream/filamentation, 512 x 512 periodic mesh,
dx = 0.2, 256 particles per cell (67,108,864 electrons), beams u_x = +-1.0 with spread
0.02, dt = 0.05, quadratic shapes, FP64, nonlinear tolerances 1e-12 (relative) / 1e-14
(absolute), beside the FP32-bulk mode.  Inputs are seeded synthetic arrays, resident in
HBM before timing.

One timed step is one full implicit Crank-Nicolson step (all outer iterations, each
with the field solve, the orbit pass with its inner Picard loop and the deposit).
`value` counts particle orbit evaluations (one particle through one Picard
iteration of the orbit pass) per second of wall time over the timed steps.

The JSON line also carries the roofline of the dominant kernel (the orbit pass) from
its HIP-event timed launches, the FP32-bulk mode (at its own tolerances, and FP64 at
those same tolerances, so the gain from precision and the gain from the looser tests
are stated apart), an on-device copy bandwidth, and the CPU oracle's rate on a bounded
sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s per Picard iter (FP64 vs FP32-bulk) at ΔE/E≤1e-6; %HBM peak"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VALU_TFLOPS = 78.6
# orbit launches are timed on every TIMING_EVERY-th step of the timed region
TIMING_EVERY = 4


def flops_per_eval(d, seg_mean, ngl, shape=2):
    """Algorithmic flops of one orbit evaluation (FMA = 2, a square root or a divide = 1).

    Quadratic shape S_2 (3 support nodes per axis), per Gauss-Legendre point:
    - gathers, per support node: grad phi (d), the D_i A sums of A^n and A^{n+1} (6d) and
      the S-bar accumulation of the orbit current (1), so 2 * 3^d * (7d + 1);
    - weights: 1D values and derivatives (20 per axis), their tensor products (0, 27, 120
      for d = 1, 2, 3) and the time blend (6 per axis).
    Per evaluation: seg * n_GL points, the endpoint interpolant A^+ (2 * 3 * 3^d gathers
    plus one point's weights without the blend) and the push, HC rotation, secant
    velocity and inner test (250).  The deposit is the S-bar term of the gathers.

    The linear shape S_1 counts the same terms over 2 nodes per axis, with 6 flops per
    axis for its 1D weights (values only; the derivatives are constant on a knot segment)
    and 0, 12, 44 tensor products.
    """
    k, w1 = (3, 20) if shape == 2 else (2, 6)
    tensor = ((0, 27, 120) if shape == 2 else (0, 12, 44))[d - 1]
    point = 2 * k ** d * (7 * d + 1) + w1 * d + tensor + 6 * d
    endpoint = 2 * 3 * k ** d + w1 * d + tensor
    return seg_mean * ngl * point + endpoint + 250


def bytes_per_particle(d, bulk=8):
    """Algorithmic HBM bytes per particle per orbit launch: read x (FP64), P, q, v_in;
    write v_out, x^{n+1} (FP64), P^{n+1}.  bulk = bytes of the bulk type (8 FP64, 4 FP32)."""
    return 8 * d + 3 * bulk + bulk + 3 * bulk + 3 * bulk + 8 * d + 3 * bulk


def bytes_per_node(d):
    """Mesh bytes per node per launch: read grad phi (d), A^n, A^{n+1}, U (9);
    read-modify-write of the deposited current (3)."""
    return 8 * (d + 9) + 8 * 3 * 2


def measured_traffic(workload, dtype, shape=2):
    """HBM bytes per orbit launch from the committed counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel), or None when there is none or
    the kernel sources have changed since the counters were taken."""
    import hashlib
    tag = "" if shape == 2 else "_linear"
    path = os.path.join(ROOT, "profiles", f"k_orbit_{workload}{tag}_{dtype}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    meta = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            meta[k.strip()] = v.strip()
    if "kernel_sources" not in meta or "traffic_bytes_per_launch" not in meta:
        return None
    h = hashlib.sha256()
    for f in meta["kernel_sources"].split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != meta.get("kernel_sources_sha256"):
        return None
    return float(meta["traffic_bytes_per_launch"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, cfg_dict, ngl, parts, shape=2, sample=65536, block=1 << 24):
    """The CPU oracle's rate on the same workload: one orbit evaluation (a particle through
    one Picard iteration of the orbit pass, with its deposit) of each particle of the first
    `block` particles in load order (whole rows of cells), at frozen smooth fields of the
    workload's mesh, at the GPU's Gauss-Legendre order on all host threads; beside it a
    seeded sample of `sample` particles on one thread at the same order and at the paper's
    GL8."""
    import oracle as O
    from paper_2609_36383_amd import workloads as W

    x, u, q = parts
    d = w["dim"]
    gphi, An, Anp1, _ = W.random_fields(d, w["n"], w["length"], seed=31, amp=0.3)
    Uh = (Anp1 - An) / w["dt"]
    P = np.abs(q)[None, :] * u
    v = u / np.sqrt(1.0 + (u * u).sum(axis=0))[None, :]

    def rate(idx, order, threads):
        sim = O.OracleSim(O.config_from_dict(cfg_dict, gl_order=order, shape_order=shape, threads=threads))
        xs, us, qs = (x, u, q) if idx is None else (x[:, idx], u[:, idx], q[idx])
        Ps, vs = (P, v) if idx is None else (P[:, idx], v[:, idx])
        sim.load_particles(xs, us, qs)
        sim.set_particle_state(xs, Ps, vs)
        t0 = time.perf_counter()
        sim.orbit_pass(gphi, An, Anp1, Uh, vs, iterate=False)
        el = time.perf_counter() - t0
        return qs.size / el, el

    threads = int(O.lib().orc_max_threads())
    nb = min(block, q.size)
    full, el = rate(None if nb == q.size else np.arange(nb), ngl, 0)
    idx = np.sort(np.random.default_rng(53).choice(q.size, min(sample, q.size), replace=False))
    one, el1 = rate(idx, ngl, 1)
    one8, el8 = rate(idx, 8, 1)
    return {"value": full, "unit": "particle-iterations/s", "cores": threads, "kind": "oracle",
            "single_thread": one, f"single_thread_gl8": one8,
            "host": f"{_cpu_model()}, nproc {os.cpu_count()}",
            "sample": f"one frozen-field orbit evaluation with deposit of {nb} of the {q.size} particles (the first "
                      f"in load order, GL{ngl} per knot segment, the GPU's order) in {el:.1f} s on {threads} OpenMP "
                      f"threads; a seeded sample of "
                      f"{idx.size} particles on 1 thread: {one:.4g}/s at GL{ngl} ({el1:.1f} s), {one8:.4g}/s at "
                      f"GL8 ({el8:.1f} s)"}


def copy_bandwidth():
    """Device-to-device copy bandwidth on this GPU (read + write bytes per second of a
    2 GiB FP64 copy, best of five), the practical ceiling beside the 8 TB/s datasheet."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * n * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def copy_probe():
    """One 256 MiB FP64 device copy: reads and writes 2^28 bytes each, the reference
    against which the profiler's FETCH_SIZE / WRITE_SIZE counters are scaled."""
    import torch
    n = 1 << 25
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}), flush=True)


PEAK_FP32_VALU_TFLOPS = 157.3


def run_case(args, w, fp32, parts, tol_of_fp32=None):
    """Time args.steps whole implicit steps of workload w in one precision mode (with
    tol_of_fp32, at the tolerances of that mode instead of its own)."""
    import torch

    from paper_2609_36383_amd import gmhc as G
    from paper_2609_36383_amd import workloads as W

    base = W.config_dict(w, fp32_bulk=fp32 if tol_of_fp32 is None else tol_of_fp32)
    sh = args.shape
    ngl = args.gl_order if args.gl_order else (w["dim"] + 1 if sh == 2 else (w["dim"] + 2) // 2)
    # the orbit launches of every TIMING_EVERY-th step record HIP events (the events
    # leave small gaps on the stream, so they stay off the other steps)
    cfg = G.config_from_dict(base, gl_order=ngl, sort_every=args.sort_every,
                             timing=TIMING_EVERY if args.steps >= TIMING_EVERY else 1,
                             precision=G.FP32_BULK if fp32 else G.FP64, shape_order=sh)
    x, u, q = parts
    npart = q.size
    sim = G.Simulation(cfg, npart, device="cuda:0")
    sim.load_particles(x, u, q)
    pot = W.potentials(w)
    if pot is not None:
        sim.load_potentials(*pot)
    sim.initialize()
    # relative energy drift, max over the sampled states: every warmup step and the
    # state after the timed steps (diagnostics stay outside the timed region)
    drift = 0.0
    for _ in range(args.warmup):
        sim.step()
        drift = max(drift, sim.diagnostics()["energy_rel"])
    torch.cuda.synchronize()
    evals = timed_evals = orbit_ms = 0.0
    launches = timed_launches = outer = segs = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rep = sim.step()
        evals += rep["evaluations"]
        orbit_ms += rep["orbit_ms"]
        launches += rep["orbit_launches"]
        if rep["orbit_ms"] > 0.0:
            timed_launches += rep["orbit_launches"]
            timed_evals += rep["evaluations"]
        outer += rep["outer_iters"]
        segs += rep["segments"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    drift = max(drift, sim.diagnostics()["energy_rel"])
    del sim
    d = w["dim"]
    ng = int(np.prod(w["n"]))
    seg_mean = segs / max(evals, 1)  # measured knot-split segments per evaluation
    # flops of the timed launches (evaluations per launch of the timed steps)
    flops_launch = (timed_evals / max(timed_launches, 1)) * flops_per_eval(d, seg_mean, ngl, sh)
    bytes_launch = npart * bytes_per_particle(d, 4 if fp32 else 8) + ng * bytes_per_node(d)
    launch_s = (orbit_ms / max(timed_launches, 1)) * 1e-3
    peak = PEAK_FP32_VALU_TFLOPS if fp32 else PEAK_FP64_VALU_TFLOPS
    achieved = flops_launch / launch_s / 1e12
    gbs = bytes_launch / launch_s / 1e9
    return dict(
        value=evals / elapsed, ms_per_step=elapsed * 1e3 / args.steps, ngl=ngl, npart=npart,
        ns_per_evaluation=launch_s * 1e9 / max(timed_evals / max(timed_launches, 1), 1),
        particle_steps_per_s=npart * args.steps / elapsed, outer_iters_mean=outer / args.steps,
        evaluations_per_particle_step=evals / (npart * args.steps), energy_drift=drift,
        segments_per_evaluation=seg_mean,
        tolerances={k: base[k] for k in ("tol_outer_rel", "tol_outer_abs", "tol_inner_rel", "tol_inner_abs")},
        roofline={
            "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(args.workload, "fp32" if fp32 else "fp64", sh),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "kernel": f"k_orbit<{d}, {sh}, {ngl}, {'float' if fp32 else 'double'}, false>", "launch_ms": launch_s * 1e3,
            "flops_per_launch": flops_launch, "hbm_bytes_per_launch": bytes_launch,
            "hbm_achieved_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS,
            # the published FP32 peak counts packed instructions, which this build does not
            # emit; non-packed FP32 issues at the FP64 rate
            **({"frac_of_nonpacked_fp32": achieved / (PEAK_FP32_VALU_TFLOPS / 2)} if fp32 else {}),
        })


def adjoint_block():
    """Gradient of the final field energy with respect to the eight perturbation amplitudes
    and the beam momentum on the 1D adjoint workload (1024 cells, 1,048,576 particles, 50
    steps, checkpoints every 10): wall times of the forward run and of the backward pass
    (re-run of each checkpoint segment, then the adjoint steps)."""
    import torch

    from paper_2609_36383_amd import adjoint as A
    from paper_2609_36383_amd import gmhc as G
    from paper_2609_36383_amd import workloads as W

    w = W.spec("tsi1d_big")
    steps, every = 50, 10
    cfg = G.config_from_dict(W.config_dict(w), sort_every=1)  # sorted every step, as the forward line
    eps = torch.full((len(w["modes"]),), w["eps"], dtype=torch.float64, requires_grad=True)
    u0 = torch.tensor(w["u_drift"], dtype=torch.float64, requires_grad=True)
    x, u, q = A.quiet1d_inputs(w, eps, u0)
    out = _time_adjoint(lambda: A.field_energy_run(x, u, q, cfg, steps, every, "cuda:0"), w["num_particles"], steps,
                        (eps, u0))
    out["workload"] = f"tsi1d_big: 1024 cells, {w['num_particles']} particles, {steps} steps, checkpoints every {every}, FP64"
    out["grad_eps"] = [float(v) for v in eps.grad]
    out["grad_u0"] = float(u0.grad)
    return out


def adjoint_block_2d():
    """The same on the 2D Weibel workload (128 x 128, 1,048,576 particles), 20 steps with
    checkpoints every 10: gradient of the final field energy with respect to every
    particle's position, momentum and charge (reported: the derivative along the beam drift)."""
    import torch

    from paper_2609_36383_amd import adjoint as A
    from paper_2609_36383_amd import gmhc as G
    from paper_2609_36383_amd import workloads as W

    w = W.spec("weibel2d")
    steps, every = 20, 10
    cfg = G.config_from_dict(W.config_dict(w), sort_every=1)  # sorted every step, as the forward line
    x, u, q = W.particles(w)
    xt = torch.tensor(x, requires_grad=True)
    ut = torch.tensor(u, requires_grad=True)
    qt = torch.tensor(q, requires_grad=True)
    out = _time_adjoint(lambda: A.field_energy_run(xt, ut, qt, cfg, steps, every, "cuda:0"), w["num_particles"], steps,
                        (xt, ut, qt))
    out["workload"] = f"weibel2d: 128x128 mesh, {w['num_particles']} particles, {steps} steps, checkpoints every {every}, FP64"
    out["grad_drift"] = float((ut.grad[2] * torch.sign(ut.detach()[2])).sum())
    return out


def adjoint_block_3d():
    """The same on the paper's 3D two-stream run TSI-0.1 (32^3 mesh, 655,360 particles,
    eigenmode start), 10 steps with checkpoints every 5 (reported: the derivative along the
    beam speed)."""
    import torch

    from paper_2609_36383_amd import adjoint as A
    from paper_2609_36383_amd import gmhc as G
    from paper_2609_36383_amd import workloads as W

    w = W.spec("tsi")
    steps, every = 10, 5
    cfg = G.config_from_dict(W.config_dict(w), sort_every=1)  # sorted every step, as the forward line
    x, u, q = W.particles(w)
    xt = torch.tensor(x, requires_grad=True)
    ut = torch.tensor(u, requires_grad=True)
    qt = torch.tensor(q, requires_grad=True)
    out = _time_adjoint(lambda: A.field_energy_run(xt, ut, qt, cfg, steps, every, "cuda:0"), w["num_particles"], steps,
                        (xt, ut, qt))
    out["workload"] = f"tsi (TSI-0.1): 32^3 mesh, {w['num_particles']} particles, {steps} steps, checkpoints every {every}, FP64"
    out["grad_beam_speed"] = float((ut.grad[0] * torch.sign(ut.detach()[0])).sum())
    return out


def _time_adjoint(run, n, steps, leaves):
    import torch
    # one untimed forward and backward pass first (kernel loads and first allocations), as
    # the forward line's warm-up steps; its gradients are dropped (the graph of the inputs is
    # kept for the timed pass)
    run().backward(retain_graph=True)
    for t in leaves:
        t.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Wt = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Wt.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fn = Wt.grad_fn
    its = [r["iterations"] for r in fn.reports]
    return {
        "field_energy": float(Wt.detach()),
        "forward_s": t1 - t0,
        "backward_s": t2 - t1,
        "backward_rerun_s": fn.seconds["rerun"],
        "backward_adjoint_steps_s": fn.seconds["adjoint_steps"],
        "ms_per_adjoint_step": 1e3 * fn.seconds["adjoint_steps"] / steps,
        "adjoint_particle_steps_per_s": n * steps / fn.seconds["adjoint_steps"],
        "transposed_outer_iterations_mean": float(np.mean(its)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed2d")
    ap.add_argument("--sort-every", type=int, default=1,
                    help="steps between particle sorts (1: every step, which keeps the workgroups' "
                         "particles within a cell or two and pays for itself at these sizes)")
    ap.add_argument("--gl-order", type=int, default=0)
    ap.add_argument("--shape", type=int, choices=(1, 2), default=2,
                    help="particle-shape B-spline degree: 2 quadratic (the paper's), 1 linear")
    ap.add_argument("--precision", choices=("both", "fp64", "fp32"), default="both",
                    help="FP64 (the headline value), FP32-bulk, or both (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint block (gradient of the 1D run's final field energy)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint block and print it as one JSON line (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 256 MiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_block(), "adjoint_2d": adjoint_block_2d(),
                          "adjoint_3d": adjoint_block_3d()}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the orbit pass on a single MI355X "
              "(multi-GPU sharding is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2609_36383_amd import workloads as W

    w = W.spec(args.workload)
    parts = W.particles(w)
    main_fp32 = args.precision == "fp32"
    r = run_case(args, w, main_fp32, parts)
    other = run_case(args, w, True, parts) if args.precision == "both" else None
    matched = run_case(args, w, False, parts, tol_of_fp32=True) if args.precision == "both" else None
    copy_gbs = copy_bandwidth()
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "particle-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-bulk" if main_fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {'x'.join(map(str, w['n']))} mesh, {r['npart']} particles, "
                               f"{w['ppc']} per cell, dt {w['dt']}, GL{r['ngl']} per knot segment"
                               + ("" if args.shape == 2 else ", linear B-spline shape")
                               + f", particles sorted every {args.sort_every} step(s)",
                   "global_batch": r["npart"], "seq_len": None, "parallelism": "single GPU"},
    }
    for k in ("particle_steps_per_s", "outer_iters_mean", "evaluations_per_particle_step", "energy_drift",
              "segments_per_evaluation", "tolerances"):
        out[k] = r[k]
    out["ns_per_evaluation"] = r["ns_per_evaluation"]
    out["roofline"] = r["roofline"]
    out["roofline"]["hbm_copy_gbs"] = copy_gbs
    out["roofline"]["hbm_frac_of_copy"] = r["roofline"]["hbm_achieved_gbs"] / copy_gbs
    if other is not None:
        keys = ("value", "ms_per_step", "particle_steps_per_s", "outer_iters_mean", "evaluations_per_particle_step",
                "energy_drift", "ns_per_evaluation", "tolerances", "roofline")
        f = out["fp32_bulk"] = {k: other[k] for k in keys}
        f["unit"] = "particle-iterations/s"
        # the gain of FP32-bulk, split: the same tolerances in both precisions (the gain
        # from precision alone), per orbit evaluation in the kernel, and with each mode's
        # own tolerances (which adds the gain of fewer outer and inner iterations)
        f["fp64_at_fp32_tolerances"] = {k: matched[k] for k in keys if k != "roofline"}
        f["speedup_per_evaluation_vs_fp64"] = r["ns_per_evaluation"] / other["ns_per_evaluation"]
        f["speedup_particle_steps_same_tolerances"] = other["particle_steps_per_s"] / matched["particle_steps_per_s"]
        f["speedup_particle_steps_own_tolerances"] = other["particle_steps_per_s"] / r["particle_steps_per_s"]
        f["speedup_per_iteration_vs_fp64"] = other["value"] / r["value"]
    if not args.no_adjoint:
        out["adjoint"] = adjoint_block()
        out["adjoint_2d"] = adjoint_block_2d()
        out["adjoint_3d"] = adjoint_block_3d()
    if not args.no_cpu_baseline:
        base = W.config_dict(w, fp32_bulk=main_fp32)
        out["cpu_baseline"] = cpu_baseline(w, base, r["ngl"], parts, shape=args.shape)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
