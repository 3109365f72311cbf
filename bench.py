"""Benchmark of the MRCM Darcy step on one MI355X.

One step = one pass of the whole hot path on one batch of synthetic input:
update the mobility from a saturation field already resident in HBM,
assemble and solve every subdomain's Robin problems for all basis
functions, solve the FP64 interface system, compose the pressure, stitch
the fine flux and check mass conservation (outputs written to device
memory).  Default workload: 1024 x 1024 cells, 4096 subdomains of 16 x 16
cells, log-normal permeability (variance 6, correlation length 0.05),
two-phase mobility with viscosity ratio 10, linear interface spaces,
alpha = 1.  ``--workload channel2048x1024`` runs the 2048 x 1024 channelized
case with 32 x 32 subdomains.

Prints one JSON line (see the keys below).  The CPU oracle is timed on a
bounded sample: one full step of the same workload on one core, and one
step per worker of a process pool over all cores (different saturation
snapshots), before the GPU is touched.  The implicit transport step
(Newton + BiCGSTAB on the GPU) and the sequential implicit step (transport
+ Darcy) are timed after the Darcy forms, on the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MRCM Darcy ms/step, subdomain solves/s @1024²: FP64 vs FP32+IR vs surrogate"

# Algorithmic work of the local problem of an m x m subdomain in the
# tile-sparse form (block-tridiagonal factorisation; 17-column solve),
# FLOP: 0.179 M and 0.418 M at m = 16; the factorisation grows as m^4 and
# the solve as m^3 (12.6 GFLOP per step for 2048 subdomains of 32 x 32).
FLOP_FACTOR_16 = 0.179e6
FLOP_SOLVE17_16 = 0.418e6
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# BF16 network: 3x3 convolutions 5->32->32->32->16 on 256 cells, 2 FLOP per
# multiply-add over the real (unpadded) channels
CNN_FLOP_PATCH = 2 * 256 * 9 * (5 * 32 + 32 * 32 + 32 * 32 + 32 * 16)
PEAK_BF16_TFLOPS = 2500.0
# transport, algorithmic HBM bytes per cell (the couplings one per face,
# about two per cell): one BiCGSTAB iteration (two fused kernels: 7 + 12
# doubles read or written per cell) and one Newton iteration outside the
# iterations (assembly 10 doubles, the solve's first p and v = A p 6,
# update 3)
TRANSPORT_BYTES_ITER = 19 * 8
TRANSPORT_BYTES_NEWTON = 19 * 8

# the roofline kernel of each subdomain size, and the sources its counter
# summary was taken on
KERNELS = {
    16: ("basis_pair_kernel<false, 4>", ("local_mfma.hip", "local_common.h", "mrcm_internal.h", "mfma_tile.h")),
    32: ("basis32x32_kernel<false, 4>", ("local_mfma32.hip", "local_common.h", "mrcm_internal.h", "mfma_tile.h")),
}


def log(*a):
    """Progress of the run on stderr (the JSON line goes to stdout)."""
    print("bench:", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gauss1024")
    ap.add_argument("--forms", default=None,
                    help="comma list of forms to time; the first one is the headline value "
                         "(default fp64,fp32_ir,surrogate; fp64,fp32_ir for 32 x 32 subdomains)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-transport", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the gravity and physics-space variants of the step")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle process pool size (default: the usable cores, at most 16)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--train-seconds", type=float, default=30.0,
                    help="surrogate form: training time budget before the timed steps")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 256 MiB device to device once before timing (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--train-fields", type=int, default=8,
                    help="surrogate form: fields (half log-normal, half channelized) whose "
                         "FP64 solves give the training patches")
    ap.add_argument("--train-snapshots", type=int, default=3,
                    help="surrogate form: saturation snapshots per training field")
    return ap.parse_args()


def traffic_file(kernel, workload):
    base = kernel.split("<")[0]
    return os.path.join(ROOT, "profiles", "hbm_traffic_%s_%s.md" % (base, workload))


def measured_traffic(kernel, sources, workload):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when it is missing or was taken on kernel sources other
    than the current ones."""
    import hashlib
    path = traffic_file(kernel, workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    csrc = os.path.join(ROOT, "paper_2104_04653_amd", "csrc")
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in sources)).hexdigest()
    if vals.get("source_sha256") != sha or vals.get("workload") != workload:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# CPU oracle timing (runs before anything touches the GPU; the pool forks)
# ---------------------------------------------------------------------------

_POOL = {}


def _oracle_step(k):
    from threadpoolctl import threadpool_limits
    import inputs
    from oracle.discretization import total_mobility
    from oracle.mrcm import solve_mrcm
    prob = _POOL["prob"]
    sat = inputs.synthetic_saturation(prob, k % prob.steps, prob.steps)
    lam = total_mobility(sat, prob.mu_w, prob.mu_o)
    phases = {}
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        solve_mrcm(prob, lam=lam, timings=phases)
        return time.perf_counter() - t0, phases


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, workers):
    """The oracle as it stands: one full step on one core, then one step per
    worker of a pool of single-threaded processes over all cores."""
    import multiprocessing as mp
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for var in saved:
        os.environ[var] = "1"
    _POOL["prob"] = prob
    usable = len(os.sched_getaffinity(0))
    P = workers if workers > 0 else max(1, min(16, usable))
    dt1, phases = _oracle_step(0)
    log("oracle, one core: %.1f s" % dt1)
    ctx = mp.get_context("fork")
    with ctx.Pool(P) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_step, range(P), chunksize=1)
        wall = time.perf_counter() - t0
    log("oracle, %d workers: %.1f s" % (P, wall))
    for var, val in saved.items():
        if val is None:
            os.environ.pop(var, None)
        else:
            os.environ[var] = val
    single = {"value": prob.n_sub / dt1, "unit": "subdomain solves/s", "cores": 1,
              "ms_per_step": 1e3 * dt1,
              "phases_ms": {k: 1e3 * v for k, v in phases.items()}}
    return {"value": P * prob.n_sub / wall, "unit": "subdomain solves/s", "cores": P,
            "kind": "oracle",
            "sample": "%d full oracle steps of the same workload (%d subdomains each, one per "
                      "single-threaded worker, different saturation snapshots) in %.1f s wall; "
                      "SuperLU local and interface solves" % (P, prob.n_sub, wall),
            "ms_per_step_per_worker": 1e3 * sum(r[0] for r in res) / P,
            "single_core": single, "nproc": os.cpu_count(), "usable_cores": usable,
            "cpu_model": cpu_model()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the MRCM Darcy step of this build is a "
              "single-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import inputs

    prob = inputs.make_problem(args.workload, seed=args.seed)
    m = prob.sub_nx
    forms_arg = args.forms or ("fp64,fp32_ir,surrogate" if m == 16 else "fp64,fp32_ir")
    cpu = None if args.no_cpu_baseline else cpu_baseline(prob, args.cpu_workers)

    import torch
    from paper_2104_04653_amd import MRCMSolver
    from paper_2104_04653_amd.mrcm import Stats

    n_steps_total = args.warmup + args.steps
    horizon = max(prob.steps, n_steps_total)
    sats = [torch.from_numpy(inputs.synthetic_saturation(prob, k % horizon, horizon)).cuda()
            for k in range(n_steps_total)]
    p = torch.empty(prob.nx * prob.ny, dtype=torch.float64, device="cuda")
    ux = torch.empty((prob.nx + 1) * prob.ny, dtype=torch.float64, device="cuda")
    uy = torch.empty(prob.nx * (prob.ny + 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    import ctypes

    surrogate_info = {}

    def trained_surrogate():
        """Network trained on patches of FP64 solves of other fields of the
        same family (log-normal and channelized), outside the timed region."""
        from paper_2104_04653_amd import SurrogateNet, surrogate
        t0 = time.perf_counter()
        cases = []
        for k in range(args.train_fields):
            if k % 2 == 0:
                q = inputs.make_problem(args.workload, seed=1000 + k)
            else:
                q = inputs.make_problem("channel256_q5", seed=1000 + k, nx=prob.nx, ny=prob.ny)
            for j in range(args.train_snapshots):
                step = (k + 3 * j) % q.steps
                cases.append((q, inputs.synthetic_saturation(q, step, q.steps)))
        x, y = surrogate.method_patches(cases)
        t_data = time.perf_counter() - t0
        log("surrogate training data: %d patches, %.1f s" % (x.shape[0], t_data))
        net = SurrogateNet(max(512, prob.n_sub), seed=args.seed)
        n_hold = 512
        t1 = time.perf_counter()
        losses = surrogate.train(net, x[n_hold:], y[n_hold:], steps=100000, batch=256, lr=2e-3,
                                 time_limit=args.train_seconds)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        surrogate_info.update({
            "training_patches": int(x.shape[0] - n_hold), "data_s": t_data,
            "train_steps": int(len(losses)), "train_s": t_train, "batch": 256,
            "heldout_mse": surrogate.evaluate(net, x[:n_hold], y[:n_hold]),
            "train_loss_first_last": [float(losses[0]), float(losses[-1])]})
        del x, y
        return net

    last_p = {}

    def run_form(precision, variant=None):
        """Time the steps of one form; variant: (label, problem) of the same
        workload with another interface space or with gravity."""
        sol = MRCMSolver(variant[1] if variant else prob, precision=precision)
        net = None
        if precision == "surrogate":
            net = trained_surrogate()
            sol.set_surrogate(net)
        outs = [ctypes.c_void_p(t.data_ptr()) for t in (p, ux, uy)]
        satp = [ctypes.c_void_p(t.data_ptr()) for t in sats]
        imb = ctypes.c_double()
        stats = Stats()

        def step(k):
            # mobility update, solve and fine-scale reconstruction in one
            # library call (one synchronisation); the saturations are device
            # arrays on the solver's stream
            rc = sol.lib.mrcm_step(sol.ctx, satp[k], 0, 1, *outs, 1, ctypes.byref(imb))
            sol._check(rc, "mrcm_step")
            sol._check(sol.lib.mrcm_get_stats(sol.ctx, ctypes.byref(stats)), "mrcm_get_stats")
            return stats

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        phase = {"local": [], "interface": [], "flux": [], "surrogate_inference_gate": []}
        iters, fallbacks, iface_ir, imb_max = 0, 0, 0, 0.0
        t0 = time.perf_counter()
        for k in range(args.warmup, n_steps_total):
            st = step(k)
            phase["local"].append(st.ms_local)
            phase["interface"].append(st.ms_interface)
            phase["flux"].append(st.ms_flux)
            phase["surrogate_inference_gate"].append(st.ms_surrogate)
            iters = max(iters, st.ir_iters_max)
            fallbacks = max(fallbacks, st.fallbacks)
            iface_ir = max(iface_ir, st.interface_ir_steps)
            imb_max = max(imb_max, imb.value)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_dof = sol.n_dof
        iface_gflop, iface_launches = stats.interface_gflop, stats.interface_launches
        last_p[precision] = (p.clone(), torch.cat([ux, uy]))
        extra = {}
        if net is not None:
            extra["training"] = dict(surrogate_info)
            extra["cnn_forward"] = cnn_forward_rate(net, sol)
            net.close()
        sol.close()
        ms_step = 1e3 * dt / args.steps
        return {"ms_per_step": ms_step, "subdomain_solves_per_s": prob.n_sub / (dt / args.steps),
                "phases_ms": {k: float(np.mean(v)) for k, v in phase.items()},
                "max_cell_imbalance": imb_max, "ir_iters_max": iters,
                "fp64_fallbacks_max": fallbacks, "fallback_rate": fallbacks / prob.n_sub,
                "interface_refinement_steps_max": iface_ir,
                "interface_gflop": iface_gflop, "interface_launches": iface_launches,
                "n_dof": n_dof, **extra}

    def cnn_forward_rate(net, sol):
        """BF16 network forward on all subdomains of the last step, timed
        with events on the stream the network runs on."""
        x = sol.surrogate_inputs()
        net.forward(x)
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            net.forward(x)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.mean(times))
        flop = prob.n_sub * CNN_FLOP_PATCH
        return {"ms": ms, "tflops": flop / (ms * 1e-3) / 1e12, "peak_bf16_tflops": PEAK_BF16_TFLOPS,
                "frac": flop / (ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
                "flop_per_patch": CNN_FLOP_PATCH}

    def run_transport():
        """One implicit transport step (20 CFL) from the first saturation with
        the fluxes of its own Darcy step, then SI steps (transport + Darcy)."""
        nx, ny = prob.nx, prob.ny
        M = prob.mu_o / prob.mu_w
        sol = MRCMSolver(prob, precision="fp64")
        s_new = torch.empty_like(sats[0])
        uxt, uyt = torch.empty_like(ux), torch.empty_like(uy)
        sol.step(sats[0], out=(p, uxt, uyt))
        torch.cuda.synchronize()
        sg = np.linspace(0.0, 1.0, 200001)
        fp = 2 * sg * (1 - sg) * M / (M * sg ** 2 + (1 - sg) ** 2) ** 2   # f' of f = Ms^2/(Ms^2+(1-s)^2)
        umax = max(float(uxt.abs().max()), float(uyt.abs().max()))
        dt = 20.0 * min(prob.hx, prob.hy) / (float(fp.max()) * umax)
        sol.transport_step(sats[0], s_new, uxt, uyt, dt)          # warm-up
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            st = sol.transport_step(sats[0], s_new, uxt, uyt, dt)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        n = nx * ny
        bytes_alg = n * (TRANSPORT_BYTES_ITER * st["linear_iters"] + TRANSPORT_BYTES_NEWTON * st["newton_iters"])
        gbs = bytes_alg / (ms * 1e-3) / 1e9
        out = {"dt_cfl_multiple": 20.0, "ms_per_step": ms, "newton_iters": st["newton_iters"],
               "bicgstab_iters": st["linear_iters"], "converged": bool(st["converged"]),
               "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": gbs / PEAK_HBM_GBS, "algorithmic_bytes": bytes_alg,
                            "note": "whole transport step (all its kernels and host round trips)"}}
        # sequential implicit steps: transport, then the Darcy step with the
        # new saturation (fluxes written in place)
        s = sats[0].clone()
        si_ms = []
        for _ in range(3):
            t0 = time.perf_counter()
            sol.si_step(s, s_new, p, uxt, uyt, dt)
            torch.cuda.synchronize()
            si_ms.append(1e3 * (time.perf_counter() - t0))
            s, s_new = s_new, s
        out["si_step_ms"] = float(np.median(si_ms))
        sol.close()
        return out

    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [f.strip() for f in forms_arg.split(",") if f.strip()]
    results = {}
    for f in forms:
        results[f] = run_form(f)
        log("form %s: %.3f ms/step" % (f, results[f]["ms_per_step"]))
    head = results[forms[0]]
    ms_step = head["ms_per_step"]
    value = head["subdomain_solves_per_s"]
    avg = head["phases_ms"]
    # roofline kernel: the per-subdomain basis kernel (assembly + factor +
    # 17-column solve + refinement + traces, FP64 MFMA), timed by the
    # library's clock stamps on its stream
    flop_sd = FLOP_FACTOR_16 * (m / 16) ** 4 + FLOP_SOLVE17_16 * (m / 16) ** 3
    alg_flop = prob.n_sub * flop_sd
    achieved = alg_flop / (avg["local"] * 1e-3) / 1e12
    kernel, sources = KERNELS[m]
    traffic = measured_traffic(kernel, sources, args.workload)

    def frac_of(ms, flop, peak):
        a = flop / (ms * 1e-3) / 1e12
        return {"achieved": a, "peak": peak, "unit": "TFLOP/s", "frac": a / peak}

    # the other phases against their own ceilings
    stitch_flop = prob.n_sub * (FLOP_FACTOR_16 * (m / 16) ** 4 + 2 * FLOP_SOLVE17_16 * (m / 16) ** 3 / 17)
    phases_roofline = {
        "interface": dict(bound="mfma", gflop_algorithmic=head["interface_gflop"],
                          launches=head["interface_launches"],
                          **frac_of(avg["interface"], head["interface_gflop"] * 1e9, PEAK_FP64_TFLOPS)),
        "flux": dict(bound="mfma", gflop_algorithmic=stitch_flop * 1e-9,
                     **frac_of(avg["flux"], stitch_flop, PEAK_FP64_TFLOPS)),
    }
    for f in forms:
        if f == "fp32_ir":
            r = results[f]
            r["roofline_local"] = dict(bound="mfma", dtype="f32 factorisation + f64 refinement",
                                       **frac_of(r["phases_ms"]["local"], alg_flop, PEAK_FP32_TFLOPS))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subdomain solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: %dx%d cells, %d subdomains of %dx%d, %s, two-phase mobility "
                        "(mu_o/mu_w = 10) from synthetic front saturations, %s interface spaces "
                        "(2+2 dofs), alpha 1, %d interface unknowns"
                        % (args.workload, prob.nx, prob.ny, prob.n_sub, prob.sub_nx, prob.sub_ny,
                           ("log-normal K (variance 6, correlation length 0.05, seed %d)" % args.seed)
                           if args.workload.startswith("gauss") else
                           ("channelized K (contrast 1e6, seed %d)" % args.seed),
                           "linear" if prob.space == 0 else "edge-solution", head["n_dof"]),
            "headline_form": forms[0],
        },
        "phases_ms": avg,
        "max_cell_imbalance": head["max_cell_imbalance"],
        "roofline": {
            "kernel": kernel,
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "traffic_gbs": None if traffic is None else traffic / (avg["local"] * 1e-3) / 1e9,
            "flop_per_launch": alg_flop,
        },
        "phases_roofline": phases_roofline,
        "forms": {f: results.get(f) for f in ("fp64", "fp32_ir", "surrogate")},
    }
    if "fp64" in last_p:
        rp, rf = last_p["fp64"]
        for f in forms:
            if f != "fp64":
                fp_, ff = last_p[f]
                out["forms"][f]["rel_l2_vs_fp64_last_step"] = {
                    "p": float((fp_ - rp).norm() / rp.norm()), "flux": float((ff - rf).norm() / rf.norm())}
    if not args.no_variants:
        # the rows beyond the plain step, on the same workload and inputs:
        # gravity (g dh/dy = -1, water 1, oil 0.8) and the physics-based
        # spaces with the adaptive alpha (generic kernels, 4 + 4 dof slots)
        out["variants"] = {}
        for label, vp in (("gravity", prob.replace(gravity=-1.0, rho_w=1.0, rho_o=0.8)),
                          ("physics_spaces_adaptive_alpha",
                           prob.replace(space="physics", p_dofs=4, u_dofs=4, adaptive_alpha=(1e-2, 1e2)))):
            r = run_form("fp64", (label, vp))
            out["variants"][label] = {k: r[k] for k in ("ms_per_step", "subdomain_solves_per_s", "phases_ms",
                                                        "max_cell_imbalance", "n_dof")}
            log("variant %s: %.3f ms/step" % (label, r["ms_per_step"]))
    if not args.no_transport:
        out["transport"] = run_transport()
        log("transport: %.2f ms/step" % out["transport"]["ms_per_step"])
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
