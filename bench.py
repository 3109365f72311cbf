"""Benchmark of the MRCM Darcy step on one MI355X.

One step = one pass of the whole hot path on one batch of synthetic input:
update the mobility from a saturation field already resident in HBM,
assemble and solve every subdomain's Robin problems for all basis
functions, solve the FP64 interface system, compose the pressure, stitch
the fine flux and check mass conservation (outputs written to device
memory).  Workload: 1024 x 1024 cells, 4096 subdomains of 16 x 16 cells,
log-normal permeability (variance 6, correlation length 0.05), two-phase
mobility with viscosity ratio 10, linear interface spaces, alpha = 1.

Prints one JSON line (see the keys below).  The CPU oracle is timed on a
bounded sample (one full step of the same workload, single-threaded).
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

# Algorithmic work per subdomain of the 16x16 local problem (block-tridiagonal
# factorisation in 16x16 tiles + 17-column solve), in FLOP.
FLOP_FACTOR_SD = 0.179e6
FLOP_SOLVE17_SD = 0.418e6
PEAK_FP64_TFLOPS = 78.6
# BF16 network: 3x3 convolutions 5->32->32->32->16 on 256 cells, 2 FLOP per
# multiply-add over the real (unpadded) channels
CNN_FLOP_PATCH = 2 * 256 * 9 * (5 * 32 + 32 * 32 + 32 * 32 + 32 * 16)
PEAK_BF16_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gauss1024")
    ap.add_argument("--forms", default="fp64,fp32_ir,surrogate",
                    help="comma list of forms to time; the first one is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_basis_pair_gauss1024.md")
KERNEL_SOURCES = ("local_mfma.hip", "local_common.h", "mrcm_internal.h")


def measured_traffic(workload):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None when it is missing, for another workload, or was taken
    on kernel sources other than the current ones."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    csrc = os.path.join(ROOT, "paper_2104_04653_amd", "csrc")
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                  for f in KERNEL_SOURCES)).hexdigest()
    if vals.get("source_sha256") != sha or vals.get("workload") != workload:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(prob, sat):
    """Time the CPU oracle (as it stands) on one full step, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle.discretization import total_mobility
    from oracle.mrcm import solve_mrcm
    lam = total_mobility(sat, prob.mu_w, prob.mu_o)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        solve_mrcm(prob, lam=lam)
        dt = time.perf_counter() - t0
    return {"value": prob.n_sub / dt, "unit": "subdomain solves/s", "cores": 1,
            "kind": "oracle",
            "sample": "one full oracle step of the same workload (%d subdomains, %.1f s, "
                      "SuperLU local and interface solves, single thread)" % (prob.n_sub, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the MRCM Darcy step of this build is a "
              "single-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import inputs
    from paper_2104_04653_amd import MRCMSolver
    from paper_2104_04653_amd.mrcm import Stats

    prob = inputs.make_problem(args.workload, seed=args.seed)
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

    def run_form(precision):
        sol = MRCMSolver(prob, precision=precision)
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
        iters, fallbacks, iface_ir = 0, 0, 0
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
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_dof = sol.n_dof
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
                "max_cell_imbalance": imb.value, "ir_iters_max": iters,
                "fp64_fallbacks_max": fallbacks, "fallback_rate": fallbacks / prob.n_sub,
                "interface_refinement_steps_max": iface_ir,
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

    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {f: run_form(f) for f in forms}
    head = results[forms[0]]
    ms_step = head["ms_per_step"]
    value = head["subdomain_solves_per_s"]
    avg = head["phases_ms"]
    # roofline kernel: the per-subdomain basis kernel (assembly + factor +
    # 17-column solve + refinement + traces, FP64 MFMA), timed by the
    # library's HIP events on its stream
    alg_flop = prob.n_sub * (FLOP_FACTOR_SD + FLOP_SOLVE17_SD)
    achieved = alg_flop / (avg["local"] * 1e-3) / 1e12
    traffic = measured_traffic(args.workload)
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
            "workload": "%s: %dx%d cells, %d subdomains of %dx%d, log-normal K (variance 6, "
                        "correlation length 0.05, seed %d), two-phase mobility (mu_o/mu_w = 10) "
                        "from synthetic front saturations, linear interface spaces (2+2 dofs), "
                        "alpha 1, %d interface unknowns"
                        % (args.workload, prob.nx, prob.ny, prob.n_sub, prob.sub_nx, prob.sub_ny,
                           args.seed, head["n_dof"]),
            "headline_form": forms[0],
        },
        "phases_ms": avg,
        "max_cell_imbalance": head["max_cell_imbalance"],
        "roofline": {
            "kernel": "basis_pair_kernel",
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "traffic_gbs": None if traffic is None else traffic / (avg["local"] * 1e-3) / 1e9,
        },
        "forms": {"fp64": results.get("fp64"), "fp32_ir": results.get("fp32_ir"),
                  "surrogate": results.get("surrogate")},
    }
    if "fp64" in last_p:
        rp, rf = last_p["fp64"]
        for f in forms:
            if f != "fp64":
                fp, ff = last_p[f]
                out["forms"][f]["rel_l2_vs_fp64_last_step"] = {
                    "p": float((fp - rp).norm() / rp.norm()), "flux": float((ff - rf).norm() / rf.norm())}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, sats[0].cpu().numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
