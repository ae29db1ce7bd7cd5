"""Benchmark of the sparse SCF hot path on one MI355X.

A step is one SCF iteration of the library (Fock build, C^T H C, rotation
selection and application, re-orthonormalization, charges, energy) on the
12,288-atom synthetic water box (4096 molecules, 24,576 AOs, 16,384 occupied
MOs), inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config water4096] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SCF steps/sec + HBM GB/s at 12k atoms; FP32 vs FP64 form at 1e-6 Ha"
PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32": 157.3}   # GB/s, TFLOP/s (MI355X, dense)
# Measured HBM traffic per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel);
# it is reported only while the kernel source is the one the counters were taken from.
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_water4096_fp64.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1402_2880_amd", "csrc", "sscf_kernels.hip")
KERNEL_OF_CLASS = {"ortho_update": "sscf::k_ortho_update<6>", "spmm_tiles": "sscf::k_spmm_row<6, double>",
                   "pair_overlap": "sscf::k_pair<3, 3>", "pair_fock": "sscf::k_pair<2, 2>",
                   "rotations": "sscf::k_givens_rb<6, double>"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(system, budget_s: float, eps: float, e_conv: float):
    """The FP64 oracle on the host cores: set-up untimed, then SCF steps until the budget."""
    from oracle.oracle import Oracle
    threads = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        threads = min(threads, int(omp))
    o = Oracle(system, eps=eps, e_conv=e_conv, n_threads=threads)
    n, t_sum = 0, 0.0
    while t_sum < budget_s and n < 20:
        t = time.time()
        o.step()
        t_sum += time.time() - t
        n += 1
    return dict(value=n / t_sum, unit="SCF steps/s", cores=threads, kind="oracle",
                sample=f"oracle SCF steps 1..{n} of the same {system.name} system (set-up not timed), "
                       f"{t_sum:.1f} s")


def step_traffic(kstats, elapsed_s: float, steps: int, config: str, precision: str, seed: int):
    """HBM traffic of the timed steps: each profiled kernel's measured bytes per launch times its
    launches in the timed window (the five MFMA / gather kernels; the rest move < 5% of the
    bytes), or None when the counter summary does not match the kernel source."""
    if kstats is None:
        return None
    per = {k: measured_traffic(k, config, precision, seed) for k in KERNEL_OF_CLASS}
    if any(v is None for v in per.values()):
        return None
    total = sum(per[k] * kstats[k]["launches"] for k in per if k in kstats)
    return dict(gb_per_step=round(total / steps, 2), gb_per_s=round(total / elapsed_s, 1),
                kernels=sorted(per), source="profiles/traffic_water4096_fp64.json")


def measured_traffic(kclass: str, config: str, precision: str, seed: int):
    """HBM bytes per launch of the kernel class from the committed counter summary, or None."""
    import hashlib
    # the counters were taken on water4096 seed 1 in the FP64 form: no other workload uses them
    if config != "water4096" or precision != "fp64" or seed != 1 or not os.path.exists(TRAFFIC):
        return None
    rec = json.load(open(TRAFFIC))
    if hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest() != rec.get("kernel_source_sha256"):
        return None
    k = rec["kernels"].get(KERNEL_OF_CLASS.get(kclass, ""))
    return None if k is None else round(k["hbm_bytes_per_launch"] / 1e9, 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="water4096")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--eps", type=float, default=1e-5)
    ap.add_argument("--e-conv", type=float, default=1e-6)
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--schedule", default="step", choices=["step", "paper"],
                    help="step: step III after every step, |dE| < e-conv (default); paper: step III only at "
                         "set-up and after convergence, dq_max < 10 eps (section 4.1)")
    ap.add_argument("--setup-timing", action="store_true",
                    help="time the GPU atom neighbour map and constrained k-means (section 3.2), initial guess (section 3.3) and the library set-up (neighbour maps, "
                         "schedule, initial orthonormalization)")
    ap.add_argument("--adjoint", action="store_true",
                    help="a step is the forward SCF step plus the energy gradient (dE/dH0, dE/dS) at its MOs, "
                         "both inside the timed region")
    ap.add_argument("--gradient", action="store_true",
                    help="after the timed steps, time one energy-gradient evaluation (dE/dH0, dE/dS)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the SCF, copy a buffer of this size three times: a kernel of known "
                         "traffic against which hardware byte counters are scaled")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the sparse SCF path runs on one GPU; --gpus N with N > 1 is not supported "
              "(how it would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1402_2880_amd import synth
    from paper_1402_2880_amd.sscf import FP32_MIXED, FP64, SparseSCF

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {args.copy_calibration} MiB "
            f"({args.copy_calibration * 1024} KiB read and written each)")
        del src, dst
    t = time.time()
    system = synth.make_config(args.config, args.seed)
    log(f"[bench] {args.config}: {system.n_atoms} atoms, {system.n_ao} AOs, {system.n_mo} MOs "
        f"(generated in {time.time() - t:.1f} s)")
    prec = FP64 if args.precision == "fp64" else FP32_MIXED
    setup = None
    if args.setup_timing:
        import numpy as np
        from paper_1402_2880_amd.sscf import fragment_guess
        n_mol = int(system.atom_mol.max()) + 1
        first = np.searchsorted(system.atom_mol, np.arange(n_mol))
        last = np.searchsorted(system.atom_mol, np.arange(n_mol), side="right")
        nocc = np.array([int(round(system.q0[a:b].sum())) // 2 for a, b in zip(first, last)], dtype=np.int32)
        aoo = system.ao_offset()
        if int((aoo[last] - aoo[first]).max()) <= 8:
            fragment_guess(system, system.atom_mol, nocc, system.atom_group[first])      # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            fragment_guess(system, system.atom_mol, nocc, system.atom_group[first], drop=1e-13)
            setup = dict(guess_ms=round(1e3 * (time.perf_counter() - t), 2), fragments=n_mol)
        else:
            setup = dict(guess_ms=None, fragments=n_mol,
                         guess_note="molecules of more than 8 AOs: the GPU guess takes fragments of at most 8")
        # atom neighbour map (section 3.2): the pattern S and H are given on
        from paper_1402_2880_amd.sscf import atom_neighbours
        cut = synth.SK_CUTOFF * synth.BOHR_PER_ANGSTROM
        atom_neighbours(system.xyz_bohr, cut)                                            # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        nrp, _ = atom_neighbours(system.xyz_bohr, cut)
        setup.update(atom_map_ms=round(1e3 * (time.perf_counter() - t), 2), atom_map_nnz=int(nrp[-1]))
        # constrained k-means (section 3.2) on the molecules' first atoms, N_link per group
        from paper_1402_2880_amd.sscf import constrained_kmeans
        pts = system.xyz_bohr[first]
        m0 = synth.initial_means(np.random.default_rng(args.seed), pts, -(-n_mol // synth.N_LINK))
        constrained_kmeans(pts, m0, synth.N_LINK, max_iter=2)                            # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, kinfo = constrained_kmeans(pts, m0, synth.N_LINK, max_iter=100, tol=1e-4)
        setup.update(kmeans_ms=round(1e3 * (time.perf_counter() - t), 2), kmeans_iterations=kinfo["iterations"],
                     kmeans_rounds=kinfo["rounds"], kmeans_means=int(m0.shape[0]))
    t = time.time()
    g = SparseSCF(system, eps=args.eps, e_conv=args.e_conv, precision=prec, profile=not args.no_profile)
    if setup is not None:
        setup["init_ms"] = round(1e3 * (time.time() - t), 1)
        setup["includes"] = ("atom map: copy, count pass, scan, fill pass, copy back (two calls: size, then map); "
                             "kmeans: copies, up to 100 iterations of attribution rounds + centroid move, copy back; "
                             "guess: host-to-device copies, one thread per fragment, copy back, CSC assembly; "
                             "init: validation, neighbour map (GPU), pairs, rounds, uploads, initial orthonormalization")
    if args.schedule == "paper":
        from paper_1402_2880_amd.sscf import CONV_CHARGE
        g.set_control(args.eps, dq_conv=10 * args.eps, criterion=CONV_CHARGE, step_ortho=False)
    log(f"[bench] set-up + initial orthonormalization {time.time() - t:.1f} s "
        f"({g.init_info()['n_ortho_sweeps']} sweeps)")
    for k in range(args.warmup):
        si = g.step()
        if args.adjoint:
            g.energy_gradient()
        log(f"[bench] warmup {k + 1}: E {si['energy']:.10f} rot {si['n_rotations']} "
            f"{si['ms_total']:.1f} ms")
    if not args.no_profile:
        g.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(g.step())
        if args.adjoint:
            g.energy_gradient()      # includes the copy of dE/dH0 and dE/dS to host memory
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for k, si in enumerate(infos):
        log(f"[bench] step {args.warmup + k + 1}: E {si['energy']:.10f} dE {si['delta_e']:.2e} "
            f"rot {si['n_rotations']} sweeps {si['n_ortho_sweeps']} {si['ms_total']:.1f} ms "
            f"(fock {si['ms_fock']:.2f} cfc {si['ms_cfc']:.2f} sel {si['ms_select']:.2f} "
            f"rot {si['ms_rot']:.2f} ortho {si['ms_ortho']:.2f} sums {si['ms_sums']:.2f})")
    value = args.steps / elapsed
    roofline = None
    kstats = None
    if not args.no_profile:
        kstats = g.kernel_stats()
        for name, st in kstats.items():
            if st["launches"]:
                log(f"[bench] kernel {name}: {st['launches']} launches, {st['ms']:.2f} ms, "
                    f"{st['flops'] / max(st['ms'], 1e-9) / 1e9:.1f} TFLOP/s, "
                    f"{st['bytes'] / max(st['ms'], 1e-9) / 1e6:.1f} GB/s")
        # the dominant kernel by time
        name, st = max(kstats.items(), key=lambda kv: kv[1]["ms"])
        per_launch_ms = st["ms"] / max(st["launches"], 1)
        if st["flops"] > 0:
            achieved = st["flops"] / st["launches"] / (per_launch_ms * 1e-3) / 1e12
            # each class at the peak of the arithmetic it runs: FP64 matrix cores, except in the
            # FP32 form the C^T H C blocks and the products (whose H C launches are FP32; priced at
            # the FP32 peak, the lower fraction, although their S C launches stay FP64)
            fp32_class = args.precision == "fp32" and name in ("pair_fock", "spmm_tiles")
            peak = PEAK["fp32"] if fp32_class else PEAK["fp64"]
            roofline = dict(kernel=name, bound="mfma", achieved=round(achieved, 3), peak=peak,
                            unit="TFLOP/s", frac=round(achieved / peak, 4),
                            traffic=measured_traffic(name, args.config, args.precision, args.seed),
                            traffic_unit="GB per launch",
                            avg_launch_ms=round(per_launch_ms, 4), launches=st["launches"])
        else:
            achieved = st["bytes"] / st["launches"] / (per_launch_ms * 1e-3) / 1e9
            roofline = dict(kernel=name, bound="hbm", achieved=round(achieved, 1), peak=PEAK["hbm"],
                            unit="GB/s", frac=round(achieved / PEAK["hbm"], 4),
                            traffic=measured_traffic(name, args.config, args.precision, args.seed),
                            traffic_unit="GB per launch",
                            avg_launch_ms=round(per_launch_ms, 4), launches=st["launches"])
    grad = None
    if args.gradient:
        g.energy_gradient()                     # first call allocates its buffers
        torch.cuda.synchronize()
        t = time.perf_counter()
        gx, gs = g.energy_gradient()
        grad = dict(ms=round(1e3 * (time.perf_counter() - t), 3), n_val=int(gx.shape[0]),
                    includes="device kernels (untruncated Fock, H C, occupied-occupied pair blocks, "
                             "C_occ F, P and W on the pattern) + device-to-host copy of P and W + host assembly")
        log(f"[bench] gradient {grad}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle) ...")
        cpu = cpu_baseline(system, args.cpu_budget, args.eps, args.e_conv)
        log(f"[bench] CPU baseline {cpu}")
    last = infos[-1]
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "SCF steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config} seed {args.seed}: {system.n_atoms} atoms, {system.n_ao} AOs, "
                               f"{system.n_mo} MOs ({system.n_occ} occupied), {system.n_groups} MO groups; "
                               + (f"eps {args.eps}, e_conv {args.e_conv}" if args.schedule == "step" else
                                  f"paper schedule: eps {args.eps}, dq_max < {10 * args.eps}, step III at set-up "
                                  "and after convergence only")
                               + "; SCF steps "
                               f"{args.warmup + 1}..{args.warmup + args.steps}"
                               + ("; each step forward + adjoint (energy gradient, copied to the host)"
                                  if args.adjoint else ""),
                   "precision": args.precision, "schedule": args.schedule, "energy_last": last["energy"],
                   "converged_last": bool(last["converged"])},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    hbm = step_traffic(kstats, elapsed, args.steps, args.config, args.precision, args.seed)
    if hbm is not None:
        out["hbm"] = hbm
    if grad is not None:
        out["gradient"] = grad
    if setup is not None:
        out["setup"] = setup
    if kstats is not None:
        out["kernels"] = {k: dict(launches=v["launches"], ms=round(v["ms"], 3),
                                  tflops=round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                                  gbs=round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1))
                          for k, v in kstats.items() if v["launches"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
