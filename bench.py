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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gauss1024")
    ap.add_argument("--forms", default="fp64,fp32_ir",
                    help="comma list of forms to time; the first one is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    return ap.parse_args()


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

    def run_form(precision):
        sol = MRCMSolver(prob, precision=precision)
        outs = [ctypes.c_void_p(t.data_ptr()) for t in (p, ux, uy)]
        imb = ctypes.c_double()

        def step(k):
            sol.update_mobility(sats[k])
            sol.solve()
            rc = sol.lib.mrcm_fine_flux(sol.ctx, *outs, 1, ctypes.byref(imb))
            sol._check(rc, "mrcm_fine_flux")
            return sol.stats()

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        phase = {"local": [], "interface": [], "flux": []}
        iters, fallbacks = 0, 0
        t0 = time.perf_counter()
        for k in range(args.warmup, n_steps_total):
            st = step(k)
            phase["local"].append(st["ms_local"])
            phase["interface"].append(st["ms_interface"])
            phase["flux"].append(st["ms_flux"])
            iters = max(iters, st["ir_iters_max"])
            fallbacks = max(fallbacks, st["fallbacks"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_dof = sol.n_dof
        sol.close()
        ms_step = 1e3 * dt / args.steps
        return {"ms_per_step": ms_step, "subdomain_solves_per_s": prob.n_sub / (dt / args.steps),
                "phases_ms": {k: float(np.mean(v)) for k, v in phase.items()},
                "max_cell_imbalance": imb.value, "ir_iters_max": iters,
                "fp64_fallbacks_max": fallbacks, "n_dof": n_dof}

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
            "kernel": "basis_m16d4_kernel",
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": None,
        },
        "forms": {"fp64": results.get("fp64"), "fp32_ir": results.get("fp32_ir"),
                  "surrogate": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, sats[0].cpu().numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
