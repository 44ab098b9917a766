"""Benchmark: KD-MG solves/s on the 256^2 U(1) workload (beta = 10, m = 0.001,
32 Gaussian right-hand sides sharing one three-level hierarchy), mixed
precision, through the C ABI.  One step = one batched solve of all 32 rhs to
||b - D x|| / ||b|| <= 1e-10.  Also reported: the plain FP64 single-rhs GPU
solve rate, the fine Dslash bandwidth, the roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = {"workload": "2D U(1) staggered KD-MG solve", "lattice": [256, 256], "beta": 10.0,
            "mass": 0.001, "nrhs": 32, "levels": "3: 2x2 KD blocks; 4x4 aggregates n_vec 16 "
            "(32x32 complex coarse blocks); 2x2 aggregates n_vec 12", "tol": 1e-10,
            "coarsest": "CGNE tol 0.2, at most 1024 iterations",
            "gauge": "quenched heatbath, 200 sweeps"}
DIMS = (256, 256)
BETA, MASS, NRHS, NV, NV2 = 10.0, 0.001, 32, 16, 12
COARSE_MAXIT = 1024
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def gauge_field():
    from synth import u1_heatbath, config_seed
    return u1_heatbath(DIMS, BETA, 200, config_seed(DIMS[0], BETA, 0))


def starts(volume):
    from synth import gaussian_vectors, config_seed
    seed = config_seed(DIMS[0], BETA, 0)
    nc1 = (DIMS[0] // 8) * (DIMS[1] // 8) * 2 * NV
    return [gaussian_vectors(NV, volume, seed, tag=1), gaussian_vectors(NV2, nc1, seed, tag=2)], seed


# ------------------------------------------------------------------ CPU leg

def cpu_baseline_child(budget_its):
    """Runs in a subprocess that never touches the GPU: the oracle builds its
    own hierarchy for the same workload, then runs its FGCR on rhs 0 for
    `budget_its` outer iterations; the rate is extrapolated to a full solve
    from the residual reduction reached (FGCR converges geometrically)."""
    import numpy as np
    from synth import gaussian_vectors
    from oracle.staggered import Lattice
    from oracle.mg import MGParams, LevelParams, Hierarchy, Solver
    U, _ = gauge_field()
    lat = Lattice(DIMS)
    psi0, seed = starts(lat.volume)
    t0 = time.perf_counter()
    h = Hierarchy(lat, U, MASS, MGParams(levels=[LevelParams((4, 4), NV), LevelParams((2, 2), NV2)],
                                         outer_maxit=budget_its, coarse_maxit=COARSE_MAXIT), psi0)
    t_setup = time.perf_counter() - t0
    b = gaussian_vectors(NRHS, lat.volume, seed, tag=0)[0]
    t0 = time.perf_counter()
    _, info = Solver(h).solve(b, 1e-10)
    t_solve = time.perf_counter() - t0
    its = info["outer_its"]
    res = info["true_rel_resid"]
    est_its = its if res <= 1e-10 else its * math.log(1e-10) / math.log(res)
    per_solve = t_solve / its * est_its
    print(json.dumps({"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
                      "sample": "rhs 0 of 32 at 256^2; oracle hierarchy built first (setup %.1f s, "
                                "excluded like the GPU setup); %d outer FGCR iterations timed "
                                "(%.1f s, relative residual %.2e), rate extrapolated to 1e-10 "
                                "assuming geometric FGCR convergence (%.1f iterations)"
                                % (t_setup, its, t_solve, res, est_its),
                      "setup_s": t_setup, "seconds_timed": t_solve}))


def start_cpu_leg(budget_its):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    env["CUDA_VISIBLE_DEVICES"] = ""
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-child",
                             str(budget_its)], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                            text=True, env=env, cwd=ROOT)


# ------------------------------------------------------------------ GPU leg

def event_time(fn, reps):
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-its", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-rhs", type=int, default=1)
    ap.add_argument("--cpu-child", type=int, default=None)
    a = ap.parse_args()
    if a.cpu_child is not None:
        cpu_baseline_child(a.cpu_child)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (a.gpus, world), file=sys.stderr)
        return 2
    cpu = None if a.no_cpu else start_cpu_leg(a.cpu_its)

    import numpy as np
    import torch
    from paper_1801_07823_amd import kdmg
    from synth import gaussian_vectors
    kdmg.kdmg_init(0)
    U, ginfo = gauge_field()
    lat = kdmg.Lattice(DIMS, U)
    V = lat.volume
    psi0, seed = starts(V)
    params = kdmg.make_params([((4, 4), NV), ((2, 2), NV2)], coarse_maxit=COARSE_MAXIT,
                              outer_maxit=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = kdmg.Hierarchy(lat, MASS, params, psi0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("setup %.2f s" % setup_s, file=sys.stderr, flush=True)
    b = torch.from_numpy(gaussian_vectors(NRHS, V, seed, tag=0)).to("cuda")
    x = torch.empty_like(b)
    for i in range(a.warmup):
        info, _ = kdmg.kdmg_solve(h, b, x, NRHS, 1e-10, prec=kdmg.KDMG_MIXED)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        info, _ = kdmg.kdmg_solve(h, b, x, NRHS, 1e-10, prec=kdmg.KDMG_MIXED)
        print("step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = NRHS * a.steps / T
    max_res = max(i["true_rel_resid"] for i in info)
    assert all(i["converged"] for i in info) and max_res <= 1e-10

    # plain FP64 single-rhs GPU KD-MG on the same rhs, one after another
    x1 = torch.empty((1, V), dtype=torch.complex128, device="cuda")
    t64 = []
    info64 = []
    for r in range(a.fp64_rhs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf, _ = kdmg.kdmg_solve(h, b[r:r + 1].contiguous(), x1, 1, 1e-10, prec=kdmg.KDMG_FP64)
        torch.cuda.synchronize()
        t64.append(time.perf_counter() - t0)
        info64.append(inf[0])
        print("fp64 rhs %d: %.2f s" % (r, t64[-1]), file=sys.stderr, flush=True)
    fp64_rate = len(t64) / sum(t64)

    # fine Dslash bandwidth (algorithmic bytes / kernel time)
    vin64 = torch.randn((1, V), dtype=torch.complex128, device="cuda")
    vout64 = torch.empty_like(vin64)
    t_d64 = event_time(lambda: kdmg.kdmg_apply_D(lat, MASS, vin64, vout64, 1), 200)
    vin32 = torch.randn((NRHS, V), dtype=torch.complex64, device="cuda")
    vout32 = torch.empty_like(vin32)
    t_d32 = event_time(lambda: kdmg.kdmg_apply_D(lat, MASS, vin32, vout32, NRHS,
                                                prec=kdmg.KDMG_MIXED), 200)
    bytes_d64 = V * (16 + 16 + 2 * 16)
    bytes_d32 = V * NRHS * (8 + 8) + V * 2 * 4
    dslash = {"fp64_1rhs": {"GB/s": bytes_d64 / t_d64 / 1e9, "us": t_d64 * 1e6,
                            "bytes": bytes_d64},
              "mixed_32rhs": {"GB/s": bytes_d32 / t_d32 / 1e9, "us": t_d32 * 1e6,
                              "bytes": bytes_d32}}

    # dominant kernel: coarsest-level stencil apply (FP64, 32 rhs, 16^2 x 32 dofs)
    dims3, nd3 = h.level_info(2)
    n3 = int(np.prod(dims3)) * nd3
    c_in = torch.randn((NRHS, n3), dtype=torch.complex128, device="cuda")
    c_out = torch.empty_like(c_in)
    t_c = event_time(lambda: kdmg.kdmg_coarse_apply(h, 2, c_in, c_out, NRHS), 500)
    ns3 = int(np.prod(dims3))
    flops = 8.0 * 5 * nd3 * nd3 * ns3 * NRHS
    bytes_c = 16.0 * (5 * nd3 * nd3 * ns3 + 2 * NRHS * n3)
    roofline = {"kernel": "k_capply<double> (coarsest A_hat_hat apply, 16^2 x %d dofs, 32 rhs)" % nd3,
                "bound": "alu", "achieved": flops / t_c / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / t_c / 1e12 / FP64_PEAK_TFLOPS,
                "traffic": None, "us_per_launch": t_c * 1e6, "flops_per_launch": flops,
                "algorithmic_bytes_per_launch": bytes_c}

    cpu_res = None
    if cpu is not None:
        out, err = cpu.communicate(timeout=1800)
        try:
            cpu_res = json.loads(out.strip().splitlines()[-1])
        except Exception:
            cpu_res = {"error": err[-2000:]}
    res = {
        "metric": "KD-MG solves/s at 256^2 U(1) (mixed precision, 32 rhs, to 1e-10)",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": T / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp64 outer / fp32 V-cycle (fp16 links, P) / fp64 coarsest",
        "data": "synthetic", "config": WORKLOAD,
        "setup_s": setup_s,
        "max_true_rel_resid": max_res,
        "iterations": {"outer": [i["outer_its"] for i in info],
                       "level2_avg": [round(i["level_avg_its"][0], 2) for i in info],
                       "level3_avg": [round(i["level_avg_its"][1], 2) for i in info]},
        "fp64_single_rhs": {"value": fp64_rate, "unit": "solves/s", "rhs_timed": len(t64),
                            "outer_its": [i["outer_its"] for i in info64],
                            "mixed_over_fp64": value / fp64_rate},
        "dslash": dslash,
        "roofline": roofline,
        "cpu_baseline": cpu_res,
        "plaquette": ginfo["plaquette"],
    }
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
