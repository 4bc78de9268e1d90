#!/usr/bin/env python3
"""Benchmark: ILU(0)-preconditioned restarted GMRES(30) on the 3D 7-point lognormal
heterogeneous-diffusion system (128^3 = 2,097,152 unknowns, 14.6M nonzeros, sigma = 2),
solved to a 1e-8 relative FP64 residual on one MI355X, plus the HEC SpMV bandwidth.

A step is one full solve from x0 = 0 with the matrix, the ILU factor, its level
schedules and the right-hand side already resident in HBM. The setup (HEC
conversion, ILU(0), level schedules: host CSR in, hence PCIe-inclusive) is timed
separately and reported beside the step. `value` is solves per second over the K
timed steps; p50/p99 are the per-solve latencies.

Extra fields: the SpMV's achieved GB/s (algorithmic bytes, three rotating matrix
copies so the 256 MB last-level cache cannot hold the working set), the roofline
of the dominant kernel of the step, BiCGSTAB on the same system, one full solve of
the FP64 CPU oracle on one core of this host (and its CSR product on every core),
and two smaller records: the 2D Poisson 64^2 latency case and the 192^3 anisotropic
ILU(1) case solved in FP64 and in mixed precision to 1e-10.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes moved by one preconditioner solve (lower + upper launch) on the 128^3 system, measured with
# rocprofv3 FETCH_SIZE and WRITE_SIZE and scaled by the counts of a plain 1 GiB copy; valid for the kernels
# as they are -- reset to None whenever the solve kernels change until the counters are taken again.
TRSV_PAIR_TRAFFIC = 234725554  # k_trsv_grid lower + upper (profiles/gmres_ilu0_tpfa128_hbm_counters.md)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--m", type=int, default=128, help="grid edge of the 3D workload")
    p.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extra", action="store_true", help="skip the c1 (2D Poisson latency) and c4 (192^3 "
                                                              "FP64 vs mixed) records of the benchmark line")
    p.add_argument("--spmv-reps", type=int, default=50)
    p.add_argument("--workload", default="diffusion128",
                   choices=["diffusion128", "poisson64", "powerlaw", "aniso192", "serving", "ras", "iluk", "formats",
                            "amg", "copy"],
                   help="diffusion128 is the benchmark line; the others print extra records "
                        "(copy: a plain 1 GiB device copy, the reference for HBM byte counters)")
    p.add_argument("--requests", type=int, default=2000, help="serving: number of requests")
    p.add_argument("--slots", type=int, default=8, help="serving: requests in flight")
    p.add_argument("--batch-max-n", type=int, default=8192, help="serving: largest batched system")
    p.add_argument("--batch-wait", type=float, default=0.05, help="serving: longest hold of a batched launch (s)")
    p.add_argument("--loops", choices=["both", "closed", "open"], default="both",
                   help="serving: closed-loop and/or open-loop runs")
    p.add_argument("--open-rate", choices=["sequential", "closed"], default="sequential",
                   help="serving: open-loop arrivals at 0.7x the FP64 sequential-service throughput (measured "
                        "with one slot on the first 200 requests) or at 0.7x the closed-loop FP64 throughput")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_launches(fn, reps, stream):
    """Average duration of fn() over `reps` back-to-back calls, measured with HIP
    events recorded on the stream the kernels run on."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def formats_table():
    """Table 3 of the paper (SpMV speedup of ELL, HYB and HEC over a sequential CPU
    product) on synthetic stand-ins, with CSR beside them: FP64 SpMV time and GB/s on
    algorithmic bytes (12 nnz + 16 n) for each format, and the speedup over the
    oracle's CSR product on one pinned host core."""
    import torch
    import oracle as O
    from paper_1606_00545_amd import hec, synth
    dev = "cuda"
    stream = torch.cuda.current_stream()
    mats = [("3D Poisson 150^3 (the paper's 3D_Poisson)", lambda: synth.poisson3d(150)),
            ("power-law 4M (row lengths 4..512, mean 12)", lambda: synth.workload_powerlaw()[0]),
            ("circuit-like 2M (banded + 200 rows of 2000..20000)",
             lambda: synth.circuit_like(2_000_000, np.random.default_rng(6)))]
    res = []
    try:
        os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
    except (AttributeError, OSError):
        pass
    for name, mk in mats:
        t0 = time.time()
        A = mk()
        n, nnz = A.n, A.nnz
        maxrow = int(np.diff(A.Ap).max())
        log(f"[bench] formats: {name}: n={n} nnz={nnz} max row {maxrow} ({time.time() - t0:.1f}s)")
        x = np.random.default_rng(7).uniform(-1, 1, n)
        cpu = []
        for _ in range(3):
            tc = time.perf_counter()
            O.csr_spmv(n, A.Ap, A.Aj, A.Ax, x)
            cpu.append(time.perf_counter() - tc)
        t_cpu = min(cpu)
        alg = 12 * nnz + 16 * n
        row = {"matrix": name, "n": n, "nnz": nnz, "max_row": maxrow, "cpu_oracle_us": round(t_cpu * 1e6, 1)}
        xd = torch.from_numpy(x).to(dev)
        yd = torch.empty(n, dtype=torch.float64, device=dev)
        for fmt, width, coo in (("CSR", 0, False), ("ELL", maxrow, False), ("HYB", hec.WIDTH_HYB, True),
                                ("HEC", -1, False)):
            ld = (n + 255) // 256 * 256
            if fmt == "ELL" and 12 * maxrow * ld > 40e9:
                row[fmt] = {"skipped": f"the slab would hold {12 * maxrow * ld / 1e9:.0f} GB"}
                continue
            Mh = hec.hec_from_csr(A, ell_width=width, coo=coo)
            inf = hec.hec_info(Mh)
            t = time_launches(lambda: hec.hec_spmv(Mh, xd, yd), 20, stream)
            stored = 12 * inf["K"] * inf["ld"] + (16 if coo else 12) * inf["nnz_rem"] + 16 * n
            row[fmt] = {"K": inf["K"], "nnz_rem": inf["nnz_rem"], "us": round(t * 1e6, 1),
                        "alg_GBps": round(alg / t / 1e9, 1), "stored_GBps": round(stored / t / 1e9, 1),
                        "speedup_vs_cpu": round(t_cpu / t, 1)}
            log(f"[bench] formats {fmt}: {row[fmt]}")
            del Mh
        res.append(row)
        del A
    return {"formats": res, "note": "FP64 values and vectors; speedup = one-core oracle CSR SpMV time / GPU time"}


def amg_table():
    """Tables 6-7 of the paper (AMG with RS coarsening, direct interpolation and the damped
    Jacobi or the Chebyshev smoother, V-cycle, at most 8 levels, 3 + 3 sweeps) on the
    paper's 3D Poisson 50^3 and a 1000 x 1000 2D lognormal diffusion stand-in for
    ecology2: setup time, hierarchy, V-cycles to 1e-8 and solve time on the GPU; the
    oracle's V-cycle solve on one host core beside it for the 50^3 case (its pure-Python
    setup is too slow for 10^6 rows)."""
    import torch
    import oracle.amg as OA
    from paper_1606_00545_amd import hec, synth
    dev = "cuda"
    res = []
    try:
        os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
    except (AttributeError, OSError):
        pass
    mats = (("3D Poisson 50^3 (the paper's)", lambda: synth.poisson3d(50), True),
            ("2D lognormal diffusion 1000^2, sigma 2 (stand-in for ecology2)",
             lambda: synth.lognormal_tpfa((1000, 1000), 2.0, np.random.default_rng(8)), False))
    for (name, mk, cpu), smoother in ((m, sm) for m in mats for sm in ("jacobi", "chebyshev")):
        A = mk()
        xt = np.random.default_rng(9).uniform(-1, 1, A.n)
        ts = time.time()
        G = hec.amg_setup(A, smoother=smoother)
        t_setup = time.time() - ts
        info = hec.amg_info(G)
        opc = sum(info["nnz"]) / info["nnz"][0]
        Mh = hec.hec_from_csr(A)
        xd = torch.from_numpy(xt).to(dev)
        b = torch.empty_like(xd)
        hec.hec_spmv(Mh, xd, b)
        runs = []
        for _ in range(3):
            x = torch.empty_like(b)
            inf = hec.amg_solve(G, b, x, maxit=200, rtol=1e-8)
            runs.append(inf)
        best = min(runs, key=lambda r: r["seconds"])
        row = {"matrix": name, "smoother": smoother, "n": A.n, "nnz": A.nnz, "setup_s": round(t_setup, 3),
               "levels": info["levels"],
               "level_rows": info["n"], "operator_complexity": round(opc, 3), "cycles": best["iterations"],
               "rel_res": best["rel_res_true"], "gpu_solve_s": round(best["seconds"], 4),
               "ms_per_cycle": round(best["seconds"] * 1e3 / max(1, best["iterations"]), 3)}
        if cpu:
            H = OA.hierarchy(A, smoother=smoother)
            bh = b.cpu().numpy()
            tc = time.perf_counter()
            ro = OA.solve(H, bh, rtol=1e-8, maxit=200)
            t_cpu = time.perf_counter() - tc
            row.update(cpu_oracle_solve_s=round(t_cpu, 3), cpu_oracle_cycles=ro.iterations,
                       speedup_vs_cpu=round(t_cpu / best["seconds"], 2))
        log(f"[bench] amg: {row}")
        res.append(row)
    return {"amg": res, "note": "FP64; RS first pass, direct interpolation, damped Jacobi (omega 2/3) or Chebyshev "
                                "(degree 3 on [0.3 lmax, lmax], lmax the Gershgorin bound of D^-1 A), 3 + 3 sweeps, "
                                "at most 8 levels, coarsest <= 64 rows solved with its inverse"}


def main():
    args = parse()
    if args.workload != "diffusion128":
        return extra(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1606_00545_amd import hec, synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = args.m
    t0 = time.time()
    A, xt = synth.workload_diffusion3d(m, sigma=2.0, seed=2)
    log(f"[bench] workload 3D lognormal TPFA {m}^3: n={A.n} nnz={A.nnz} (generated in {time.time() - t0:.1f}s)")

    mixed = args.precision == "mixed"
    torch.cuda.synchronize()
    ts = time.time()
    Mh = hec.hec_from_csr(A, keep_f32=mixed)
    t_hec = time.time() - ts
    ts = time.time()
    F = hec.ilu_factor(A, k=0, keep_f32=mixed)
    t_ilu = time.time() - ts
    ts = time.time()
    lv = hec.level_schedule(F)
    t_lev = time.time() - ts
    li = hec.levels_info(lv)
    info_h = hec.hec_info(Mh)
    log(f"[bench] setup hec {t_hec:.2f}s ilu {t_ilu:.2f}s levels {t_lev:.2f}s "
        f"(levels L/U {li['nlev_lower']}/{li['nlev_upper']}, ELL K={info_h['K']})")

    xt_d = torch.from_numpy(xt).to(dev)
    b = torch.empty(A.n, dtype=torch.float64, device=dev)
    hec.hec_spmv(Mh, xt_d, b)  # b = A x_true
    x = torch.empty(A.n, dtype=torch.float64, device=dev)
    prec = 1 if mixed else 0

    def solve():
        return hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8, precision=prec)

    for w in range(args.warmup):
        inf = solve()
        log(f"[bench] warmup {w}: {inf['iterations']} it, rel_res {inf['rel_res_true']:.2e}, {inf['seconds']:.3f}s")
    torch.cuda.synchronize()
    lat = []
    iters = []
    tstart = time.time()
    for k in range(args.steps):
        t1 = time.time()
        inf = solve()
        lat.append(time.time() - t1)
        iters.append(inf["iterations"])
        assert inf["status"] == hec.OK and inf["rel_res_true"] <= 1e-8
    torch.cuda.synchronize()
    total = time.time() - tstart
    log(f"[bench] {args.steps} solves in {total:.3f}s; iterations {iters[0]}; last rel_res {inf['rel_res_true']:.2e}")
    ms_per_step = total / args.steps * 1e3

    # independent check of the last solution: true residual through the FP64 SpMV
    r = b.clone()
    hec.hec_spmv(Mh, x, r, -1.0, 1.0)
    rel_res = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    err_true = float(torch.linalg.norm(x - xt_d) / torch.linalg.norm(xt_d))

    # BiCGSTAB on the same resident system (one solve, for the record)
    xb = torch.empty_like(x)
    bi = hec.bicgstab_solve(Mh, F, lv, b, xb, rtol=1e-8)
    log(f"[bench] bicgstab: {bi['iterations']} it, {bi['seconds']:.3f}s")

    # ---- kernel timings (HIP events on the launch stream) ----
    n, nnz = A.n, A.nnz
    K = info_h["K"]
    copies = [Mh] + [hec.hec_from_csr(A) for _ in range(2)]
    xs = [torch.from_numpy(xt).to(dev) for _ in range(3)]
    ys = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    idx = [0]

    def spmv_rot():
        i = idx[0] % 3
        idx[0] += 1
        hec.hec_spmv(copies[i], xs[i], ys[i])

    t_spmv = time_launches(spmv_rot, args.spmv_reps, stream)
    spmv_bytes = 12 * nnz + 16 * n          # values + indices, x once, y written
    spmv_gbs = spmv_bytes / t_spmv / 1e9

    # the preconditioner solve M z = v: exactly two persistent launches (lower, then upper)
    lu_nnz = int(hec.ilu_info(F)["nnz"])
    zb = torch.empty(n, dtype=torch.float64, device=dev)
    t_trsv_l = time_launches(lambda: hec.trsv_levels(F, lv, b, zb, hec.LOWER), 20, stream)
    t_trsv_lu = time_launches(lambda: hec.trsv_levels(F, lv, b, zb, hec.LU), 20, stream)
    # algorithmic bytes of one L-then-U solve: 12 bytes (value + index) per stored factor entry, and
    # 32 bytes per row (the right-hand side read, the intermediate L^{-1} v written and read, z written)
    trsv_bytes = 12 * lu_nnz + 32 * n
    trsv_gbs = trsv_bytes / t_trsv_lu / 1e9
    it_per_solve = iters[-1]
    log(f"[bench] spmv {t_spmv * 1e6:.1f}us {spmv_gbs:.0f} GB/s; trsv L {t_trsv_l * 1e6:.1f}us; "
        f"trsv L+U {t_trsv_lu * 1e6:.1f}us")
    # share of the step spent in the triangular solves (one L-then-U solve per Arnoldi step)
    trsv_share = t_trsv_lu * it_per_solve / (ms_per_step / 1e3)

    grid = hec.levels_grid(lv)  # the wavefront kernel (7-point ILU(0) on a grid) or the level-blocked one
    kname = ("k_trsv_grid<double,false,8> + k_trsv_grid<double,true,8>" if grid else
             "k_trsv_blk<double,false,4> + k_trsv_blk<double,true,4>")
    roof = {"kernel": kname + " (one preconditioner solve: the lower and the upper launch)",
            "bound": "hbm", "achieved": round(trsv_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(trsv_gbs / HBM_PEAK_GBS, 5), "traffic": TRSV_PAIR_TRAFFIC if m == 128 else None,
            "traffic_note": "HBM bytes of one lower + one upper launch from rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                            "scaled by a plain copy's counts (profiles/gmres_ilu0_tpfa128_hbm_counters.md)",
            "bytes": trsv_bytes,
            "us": round(t_trsv_lu * 1e6, 1),
            "note": f"latency-bound: {li['nlev_lower']} + {li['nlev_upper']} dependent levels; "
                    f"the two solves are {trsv_share * 100:.0f}% of the step"}
    # the copy bandwidth of this machine in this run (1 GiB device-to-device), the practical HBM ceiling
    csrc = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    t_copy = time_launches(lambda: cdst.copy_(csrc), 10, stream)
    copy_gbs = 2 * csrc.numel() * 8 / t_copy / 1e9
    del csrc, cdst
    spmv_roof = {"kernel": "k_spmv_ell<double,double,double>", "bound": "hbm",
                 "achieved": round(spmv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(spmv_gbs / HBM_PEAK_GBS, 4), "us": round(t_spmv * 1e6, 2),
                 "bytes": spmv_bytes, "gflops": round(2 * nnz / t_spmv / 1e9, 1),
                 "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(spmv_gbs / copy_gbs, 4)}

    # latency bound of the triangular solve: the cost of one level on a solve that has nothing to
    # wait for but its own previous level, times the levels of both triangles. Wavefront kernel: one
    # tile of 8 x 8 columns, 4096 long (4110 steps, no other tile); blocked kernel: a chain (1D Poisson,
    # 4096 levels of one row in one part)
    if grid:
        Ac = synth.lognormal_tpfa((8, 8, 4096), 2.0, np.random.default_rng(2))
        what = "lower solve of one 8 x 8 x 4096 tile (4110 wavefront steps, nothing to wait for) / 4110"
    else:
        Ac = synth.poisson1d(4096)
        what = "lower solve of a 4096-row chain (one row per level, one part) / 4096"
    Fc = hec.ilu_factor(Ac, k=0)
    lvc = hec.level_schedule(Fc)
    bc = torch.ones(Ac.n, dtype=torch.float64, device=dev)
    zc = torch.empty_like(bc)
    t_chain = time_launches(lambda: hec.trsv_levels(Fc, lvc, bc, zc, hec.LOWER), 20, stream)
    t_level = t_chain / (4096 + 14 if grid else hec.levels_info(lvc)["nlev_lower"])
    lat_bound = (li["nlev_lower"] + li["nlev_upper"]) * t_level
    roof["latency"] = {"t_level_us": round(t_level * 1e6, 4),
                       "bound_us": round(lat_bound * 1e6, 1), "frac": round(lat_bound / t_trsv_lu, 4),
                       "note": "t_level = " + what}
    del Fc, lvc

    # ---- CPU oracle: one full solve of the same system on one pinned core ----
    cpu = None
    x_oracle = None
    if not args.no_cpu_baseline:
        import oracle as O
        Ah = A
        bh = b.cpu().numpy()
        cores_avail = sorted(os.sched_getaffinity(0))
        cpu_model = "unknown"
        try:  # the first processor's identification (a virtual machine may shorten the model name)
            info = {}
            with open("/proc/cpuinfo") as f:
                for l in f:
                    if not l.strip():
                        break
                    k, _, v = l.partition(":")
                    info[k.strip()] = v.strip()
            cpu_model = info.get("model name", "unknown")
            ids = [f"{k} {info[k]}" for k in ("vendor_id", "cpu family", "model", "stepping", "cpu MHz", "cache size")
                   if k in info]
            if ids:
                cpu_model += " (" + ", ".join(ids) + ")"
        except OSError:
            pass
        # the oracle is single-threaded; pin it to one core of this host
        os.sched_setaffinity(0, {cores_avail[0]})
        ts = time.time()
        Fo = O.iluk(Ah.n, Ah.Ap, Ah.Aj, Ah.Ax, 0)
        t_orc_ilu = time.time() - ts
        ts = time.time()
        ro = O.gmres(Ah, Fo, bh, restart=30, rtol=1e-8)
        t_orc = time.time() - ts
        ts = time.perf_counter()
        for _ in range(5):
            O.csr_spmv(Ah.n, Ah.Ap, Ah.Aj, Ah.Ax, xt)
        t_spmv1 = (time.perf_counter() - ts) / 5
        os.sched_setaffinity(0, set(cores_avail))
        # secondary figure: the same CSR product with the rows shared by every host core
        nthr = len(cores_avail)
        O.csr_spmv_omp(Ah.n, Ah.Ap, Ah.Aj, Ah.Ax, xt, nthr)
        ts = time.perf_counter()
        for _ in range(20):
            O.csr_spmv_omp(Ah.n, Ah.Ap, Ah.Aj, Ah.Ax, xt, nthr)
        t_spmvn = (time.perf_counter() - ts) / 20
        x_oracle = ro.x
        cpu = {"value": round(1.0 / t_orc, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"one full oracle ILU(0)-GMRES(30) solve of the same {m}^3 system from x0 = 0 to "
                         f"1e-8 ({ro.iterations} iterations, {t_orc:.2f} s, rel_res {ro.rel_res:.2e}); the "
                         f"oracle's ILU(0) setup ({t_orc_ilu:.2f} s) is not included; single thread pinned to "
                         f"one core, gcc -O3 -ffp-contract=off",
               "cpu_model": cpu_model, "host_cores_available": nthr,
               "spmv_1core": {"us": round(t_spmv1 * 1e6, 1), "GBps": round(spmv_bytes / t_spmv1 / 1e9, 2)},
               "spmv_all_cores": {"threads": nthr, "us": round(t_spmvn * 1e6, 1),
                                  "GBps": round(spmv_bytes / t_spmvn / 1e9, 2),
                                  "note": "secondary figure: the oracle's CSR product with its rows shared by "
                                          "OpenMP threads on every available host core"}}
        log(f"[bench] cpu oracle: full solve {t_orc:.2f} s ({ro.iterations} it); spmv 1 core "
            f"{t_spmv1 * 1e3:.1f} ms, {nthr} threads {t_spmvn * 1e3:.2f} ms")

    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "ILU(0)-GMRES(30) solves/s to 1e-8 rel res (HEC SpMV GB/s, p99 latency alongside)",
        "value": round(args.steps / total, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point lognormal TPFA diffusion {m}^3 (sigma=2, seed 2), ILU(0), "
                               f"GMRES(30), rtol 1e-8, x0=0",
                   "n": n, "nnz": nnz, "levels_lower": li["nlev_lower"], "levels_upper": li["nlev_upper"],
                   "precision": args.precision},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "iterations": it_per_solve,
        "us_per_iteration": round(ms_per_step * 1e3 / it_per_solve, 1),
        "rel_res": rel_res,
        "err_vs_x_true": err_true,
        "err_vs_oracle": (float(np.linalg.norm(x.cpu().numpy() - x_oracle) / np.linalg.norm(x_oracle))
                          if x_oracle is not None else None),
        "setup_s": {"hec_from_csr": round(t_hec, 3), "ilu_factor": round(t_ilu, 3),
                    "level_schedule": round(t_lev, 3), "note": "host CSR in (PCIe-inclusive)"},
        "spmv": spmv_roof,
        "trsv_us": {"lower": round(t_trsv_l * 1e6, 1), "lower_upper": round(t_trsv_lu * 1e6, 1),
                    "us_per_level": round(t_trsv_l * 1e6 / li["nlev_lower"], 3)},
        "bicgstab": {"iterations": bi["iterations"], "seconds": round(bi["seconds"], 4),
                     "rel_res": bi["rel_res_true"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if not args.no_extra:
        del copies, xs, ys
        out["c1_poisson64"] = c1_record(args)
        out["c4_aniso192_mixed"] = c4_record(args)
    print(json.dumps(out), flush=True)


def c1_record(args):
    """2D 5-point Poisson 64 x 64, ILU(0)-GMRES(30) to 1e-8 from x0 = 0: per-solve latency
    (a latency-bound case: 127 + 127 levels, every vector in cache), and the distance to
    the oracle's solution."""
    import torch
    import oracle as O
    from paper_1606_00545_amd import hec, synth
    A, xt = synth.workload_c1()
    Mh = hec.hec_from_csr(A)
    F = hec.ilu_factor(A, 0)
    lv = hec.level_schedule(F)
    bh = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    b = torch.from_numpy(bh).cuda()
    x = torch.empty_like(b)
    for _ in range(3):
        hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8)
    lat = []
    for _ in range(max(50, args.steps)):
        t = time.perf_counter()
        inf = hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8)
        lat.append(time.perf_counter() - t)
    lat = np.array(lat) * 1e3
    ro = O.gmres(A, O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0), bh, restart=30, rtol=1e-8)
    rec = {"workload": "2D 5-point Poisson 64x64 (n=4096), ILU(0), GMRES(30), rtol 1e-8, x0=0",
           "solves": len(lat), "solves_per_s": round(1e3 / lat.mean(), 1), "p50_ms": round(float(np.median(lat)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "iterations": inf["iterations"],
           "oracle_iterations": ro.iterations, "rel_res": inf["rel_res_true"],
           "err_vs_oracle": float(np.linalg.norm(x.cpu().numpy() - ro.x) / np.linalg.norm(ro.x))}
    log(f"[bench] c1: {rec}")
    return rec


def c4_record(args):
    """3D 7-point lognormal diffusion 192^3 with z transmissibilities x 1/100, ILU(1): the
    all-FP64 GMRES(30) solve against the mixed one (FP32 matrix, factor and basis inside,
    FP64 residual, dots, rotations and refinement), both to 1e-10 from x0 = 0."""
    import torch
    from paper_1606_00545_amd import hec, synth
    t0 = time.time()
    A, xt = synth.workload_diffusion3d(192, sigma=2.0, seed=4, zscale=0.01)
    t_gen = time.time() - t0
    ts = time.time()
    Mh = hec.hec_from_csr(A, keep_f32=True)
    F = hec.ilu_factor(A, k=1, keep_f32=True)
    lv = hec.level_schedule(F)
    t_setup = time.time() - ts
    xd = torch.from_numpy(xt).cuda()
    b = torch.empty_like(xd)
    hec.hec_spmv(Mh, xd, b)
    rec = {"workload": "3D 7-point lognormal TPFA 192^3 (sigma=2, seed 4), z faces x 1/100, ILU(1), GMRES(30), "
                       "rtol 1e-10, x0=0", "n": A.n, "nnz_lu": hec.ilu_info(F)["nnz"],
           "setup_s": round(t_setup, 2)}
    xs = {}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        x = torch.empty_like(b)
        hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-10, precision=prec, ir_rtol=1e-10, maxit=20000)
        inf = hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-10, precision=prec, ir_rtol=1e-10, maxit=20000)
        r = b.clone()
        hec.hec_spmv(Mh, x, r, -1.0, 1.0)
        xs[name] = x
        rec[name] = {"seconds": round(inf["seconds"], 4), "iterations": inf["iterations"],
                     "ir_steps": inf["ir_steps"], "rel_res": float(torch.linalg.norm(r) / torch.linalg.norm(b)),
                     "err_vs_x_true": float(torch.linalg.norm(x - xd) / torch.linalg.norm(xd))}
    rec["mixed"]["err_vs_fp64_solution"] = float(torch.linalg.norm(xs["mixed"] - xs["fp64"]) /
                                                 torch.linalg.norm(xs["fp64"]))
    rec["mixed_speedup"] = round(rec["fp64"]["seconds"] / rec["mixed"]["seconds"], 3)
    log(f"[bench] c4 (generated in {t_gen:.1f}s): {rec}")
    return rec


# ---------------------------------------------------------------------------- extra records

def extra(args):
    import torch

    from paper_1606_00545_amd import hec, synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {"workload": args.workload, "data": "synthetic"}
    if args.workload == "poisson64":
        A, xt = synth.workload_c1()
        Mh = hec.hec_from_csr(A)
        F = hec.ilu_factor(A, 0)
        lv = hec.level_schedule(F)
        xd = torch.from_numpy(xt).to(dev)
        b = torch.empty_like(xd)
        hec.hec_spmv(Mh, xd, b)
        x = torch.empty_like(b)
        for name, fn in (("gmres", lambda: hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8)),
                         ("bicgstab", lambda: hec.bicgstab_solve(Mh, F, lv, b, x, rtol=1e-8))):
            fn()
            lat = []
            for _ in range(max(args.steps, 20)):
                t = time.perf_counter()
                inf = fn()
                lat.append(time.perf_counter() - t)
            lat = np.array(lat) * 1e3
            out[name] = {"iterations": inf["iterations"], "rel_res": inf["rel_res_true"],
                         "solves_per_s": round(1e3 / lat.mean(), 2), "p50_ms": round(float(np.median(lat)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        out["trsv_lu_us"] = round(time_launches(lambda: hec.trsv_levels(F, lv, b, x, hec.LU), 50, stream) * 1e6, 2)
        out["n"] = A.n
    elif args.workload == "powerlaw":
        t0 = time.time()
        A, xt = synth.workload_powerlaw()
        log(f"[bench] power-law n={A.n} nnz={A.nnz} ({time.time() - t0:.1f}s)")
        n, nnz = A.n, A.nnz
        rows = []
        for width in (0, 8, 12, 16, 24):
            Mh = hec.hec_from_csr(A, ell_width=width, keep_f32=True)
            inf = hec.hec_info(Mh)
            for prec in ("f64", "f32"):
                dt = torch.float64 if prec == "f64" else torch.float32
                xd = torch.from_numpy(xt).to(dev, dt)
                yd = torch.empty(n, dtype=dt, device=dev)
                vals = hec.F64 if prec == "f64" else hec.F32
                t = time_launches(lambda: hec.hec_spmv(Mh, xd, yd, vals=vals), 20, stream)
                vb = 8 if prec == "f64" else 4
                alg = (vb + 4) * nnz + 2 * vb * n
                stored = (vb + 4) * inf["K"] * inf["ld"] + (vb + 4) * inf["nnz_rem"] + 4 * n + 2 * vb * n
                rows.append({"format": "CSR" if width == 0 else f"HEC K={inf['K']}", "values": prec,
                             "us": round(t * 1e6, 1), "alg_GBps": round(alg / t / 1e9, 1),
                             "stored_GBps": round(stored / t / 1e9, 1), "frac_hbm": round(alg / t / 1e9 / HBM_PEAK_GBS, 4),
                             "ell_fill": round((nnz - inf["nnz_rem"]) / max(1, inf["K"] * n), 3)})
                log(f"[bench] {rows[-1]}")
            del Mh
        out.update({"n": n, "nnz": nnz, "spmv": rows})
    elif args.workload == "aniso192":
        t0 = time.time()
        A, xt = synth.workload_diffusion3d(192, sigma=2.0, seed=4, zscale=0.01)
        log(f"[bench] aniso 192^3 n={A.n} nnz={A.nnz} ({time.time() - t0:.1f}s)")
        ts = time.time()
        Mh = hec.hec_from_csr(A, keep_f32=True)
        F = hec.ilu_factor(A, k=1, keep_f32=True)
        lv = hec.level_schedule(F)
        t_setup = time.time() - ts
        li = hec.levels_info(lv)
        xd = torch.from_numpy(xt).to(dev)
        b = torch.empty_like(xd)
        hec.hec_spmv(Mh, xd, b)
        res = {}
        for name, prec in (("fp64", 0), ("mixed", 1)):
            x = torch.empty_like(b)
            inf = hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-10, precision=prec, ir_rtol=1e-10,
                                  maxit=20000, check=False)
            r = b.clone()
            hec.hec_spmv(Mh, x, r, -1.0, 1.0)
            res[name] = {"status": inf["status"], "iterations": inf["iterations"], "ir_steps": inf["ir_steps"],
                         "seconds": round(inf["seconds"], 4), "rel_res": float(torch.linalg.norm(r) / torch.linalg.norm(b)),
                         "err_vs_x_true": float(torch.linalg.norm(x - xd) / torch.linalg.norm(xd))}
            log(f"[bench] {name}: {res[name]}")
        zb = torch.empty_like(b)
        zf = torch.empty(A.n, dtype=torch.float32, device=dev)
        bf = b.float()
        out.update({"n": A.n, "nnz": A.nnz, "nnz_lu": hec.ilu_info(F)["nnz"], "levels": li, "setup_s": round(t_setup, 2),
                    "solves": res,
                    "trsv_lu_us_f64": round(time_launches(lambda: hec.trsv_levels(F, lv, b, zb, hec.LU), 10, stream) * 1e6, 1),
                    "trsv_lu_us_f32": round(time_launches(lambda: hec.trsv_levels(F, lv, bf, zf, hec.LU), 10, stream) * 1e6, 1)})
    elif args.workload == "serving":
        out.update(serving(args))
    elif args.workload == "ras":
        # Sec. 2.5 inner RAS on the 128^3 system: blocks 1/8/128/1024, overlap 0/1 (Table 4-5 shape)
        A, xt = synth.workload_diffusion3d(args.m, sigma=2.0, seed=2)
        Mh = hec.hec_from_csr(A)
        xd = torch.from_numpy(xt).to(dev)
        b = torch.empty_like(xd)
        hec.hec_spmv(Mh, xd, b)
        rows = []
        for nb, ov in ((1, 0), (8, 0), (8, 1), (128, 0), (128, 1), (1024, 0), (1024, 1)):
            ts = time.time()
            F = hec.ilu_factor_ras(A, nb, ov, k=0) if (nb, ov) != (1, 0) else hec.ilu_factor(A, 0)
            lv = hec.level_schedule(F)
            t_setup = time.time() - ts
            li = hec.levels_info(lv)
            x = torch.empty_like(b)
            hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8)
            lat = []
            for _ in range(max(3, min(args.steps, 5))):
                t1 = time.time()
                inf = hec.gmres_solve(Mh, F, lv, b, x, restart=30, rtol=1e-8)
                lat.append(time.time() - t1)
            z = torch.empty_like(b)
            t_lu = time_launches(lambda: hec.trsv_levels(F, lv, b, z, hec.LU), 20, stream)
            row = {"blocks": nb, "overlap": ov, "factor_rows": hec.ilu_info(F)["n"],
                   "levels_lower": li["nlev_lower"], "levels_upper": li["nlev_upper"],
                   "iterations": inf["iterations"], "rel_res": inf["rel_res_true"],
                   "solve_ms": round(float(np.median(lat)) * 1e3, 2), "solves_per_s": round(1.0 / float(np.median(lat)), 3),
                   "trsv_lu_us": round(t_lu * 1e6, 1), "setup_s": round(t_setup, 2)}
            rows.append(row)
            log(f"[bench] ras {row}")
            del F, lv
        out.update({"n": A.n, "nnz": A.nnz, "ras": rows})
    elif args.workload == "iluk":
        # Table 4 shape: 3D Poisson 150^3 (3,375,000 rows, 23,490,000 nonzeros), ILU(k) for k = 0..3,
        # GMRES(30), BiCGSTAB and CG to 1e-8 from x0 = 0, b = A x_true
        A = synth.poisson3d(150)
        xt = np.random.default_rng(7).uniform(-1, 1, A.n)
        Mh = hec.hec_from_csr(A)
        xd = torch.from_numpy(xt).to(dev)
        b = torch.empty_like(xd)
        hec.hec_spmv(Mh, xd, b)
        rows = []
        for k in range(4):
            ts = time.time()
            F = hec.ilu_factor(A, k=k)
            lv = hec.level_schedule(F)
            t_setup = time.time() - ts
            li = hec.levels_info(lv)
            z = torch.empty_like(b)
            t_lu = time_launches(lambda: hec.trsv_levels(F, lv, b, z, hec.LU), 10, stream)
            row = {"k": k, "nnz_lu": hec.ilu_info(F)["nnz"], "levels": li["nlev_lower"], "setup_s": round(t_setup, 2),
                   "trsv_lu_us": round(t_lu * 1e6, 1)}
            for name, fn in (("gmres", lambda xx: hec.gmres_solve(Mh, F, lv, b, xx, restart=30, rtol=1e-8)),
                             ("bicgstab", lambda xx: hec.bicgstab_solve(Mh, F, lv, b, xx, rtol=1e-8)),
                             ("cg", lambda xx: hec.cg_solve(Mh, F, lv, b, xx, rtol=1e-8))):
                x = torch.empty_like(b)
                fn(x)
                t1 = time.time()
                inf = fn(x)
                row[name] = {"iterations": inf["iterations"], "seconds": round(time.time() - t1, 4),
                             "rel_res": inf["rel_res_true"]}
            rows.append(row)
            log(f"[bench] iluk {row}")
            del F, lv
        out.update({"n": A.n, "nnz": A.nnz, "iluk": rows})
    elif args.workload == "formats":
        out.update(formats_table())
    elif args.workload == "amg":
        out.update(amg_table())
    elif args.workload == "copy":
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        t = time_launches(lambda: dst.copy_(src), 5, stream)
        out.update({"bytes_read": nbytes, "bytes_written": nbytes, "us": round(t * 1e6, 1),
                    "GBps": round(2 * nbytes / t / 1e9, 1)})
    print(json.dumps(out), flush=True)


def serving(args):
    """Serving: requests (2D or 3D lognormal diffusion, n log-uniform in [1e3, 1e6],
    sigma in [0.5, 3], per-request seed). Three server configurations replay the same
    requests: FP64 with every request on its own stream ("fp64"), FP64 with small
    systems batched into persistent launches ("fp64_batched"), and mixed precision
    with batching ("mixed_batched"). Closed loop (all requests queued at t=0) gives
    throughput; open loop (Poisson arrivals at 0.7x the FP64 sequential-service
    throughput, measured with one slot on the first 200 requests; or 0.7x the
    closed-loop FP64 throughput) gives p50/p99 latency at a stated load."""
    from paper_1606_00545_amd import serve, synth

    t0 = time.time()
    specs = synth.serving_requests(args.requests)
    systems = []
    for spec in specs:
        A, xt = synth.request_system(spec)
        systems.append((spec.rid, A, A.to_scipy() @ xt))  # b = A x_true on the host (client side)
    log(f"[bench] serving: {len(systems)} requests generated in {time.time() - t0:.1f}s; "
        f"batched route n <= {args.batch_max_n}: {sum(1 for _, A, _ in systems if A.n <= args.batch_max_n)}")
    configs = (("fp64", 0, 0), ("fp64_batched", 0, args.batch_max_n), ("mixed_batched", 1, args.batch_max_n))

    def run(prec, bmax, arrivals, slots=args.slots):
        reqs = [serve.Request(rid, A, b, precision=prec, rtol=1e-8, arrival=float(t))
                for (rid, A, b), t in zip(systems, arrivals)]
        srv = serve.Server(slots=slots, batch_max_n=bmax, batch_wait=args.batch_wait)
        t = time.perf_counter()
        stop = threading.Event()

        def progress():  # a line every 30 s while a run lasts (long open-loop runs)
            while not stop.wait(30.0):
                log(f"[bench] serving: {len(srv.results)} of {len(reqs)} done after {time.perf_counter() - t:.0f} s")
        mon = threading.Thread(target=progress, daemon=True)
        mon.start()
        try:
            res = srv.run(reqs, t0=t)
        finally:
            stop.set()
            mon.join()
        span = max(r.done for r in res) if res else 0.0
        st = serve.latency_stats(res)
        ok = sum(1 for r in res if r.info["status"] == 0 and r.info["rel_res_true"] <= 1e-8)
        small = [r.latency * 1e3 for r in res if r.n <= args.batch_max_n]
        bad = [(r.rid, r.n, int(r.info["status"]), float(r.info["rel_res_true"])) for r in res
               if not (r.info["status"] == 0 and r.info["rel_res_true"] <= 1e-8)]
        return {"completed": len(res), "converged": ok, "errors": len(srv.errors),
                "solves_per_s": round(len(res) / span, 3) if span else None,
                "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
                "small_p50_ms": round(float(np.percentile(small, 50)), 2) if small else None,
                "peak_inflight": srv.peak_inflight, "batched_launches": len(srv.batches),
                "mean_batch": round(float(np.mean(srv.batches)), 1) if srv.batches else 0,
                "peak_reported_GB": round(srv.peak_reported / 1e9, 2), "not_converged": bad[:5]}

    out = {"requests": len(systems), "slots": args.slots, "batch_max_n": args.batch_max_n,
           "batch_wait_s": args.batch_wait}
    closed = {}
    for name, prec, bmax in configs if args.loops != "open" else ():
        closed[name] = run(prec, bmax, np.zeros(len(systems)))
        log(f"[bench] serving closed-loop {name}: {closed[name]}")
    out["closed_loop"] = closed
    if args.loops == "closed":
        return out
    if args.open_rate == "sequential" or not closed:  # FP64 one request at a time, on a prefix of the trace
        head = systems[:200]
        reqs = [serve.Request(rid, A, b, precision=0, rtol=1e-8, arrival=0.0) for rid, A, b in head]
        srv = serve.Server(slots=1)
        t = time.perf_counter()
        res = srv.run(reqs, t0=t)
        seq_rate = len(res) / max(r.done for r in res)
        out["sequential_fp64_solves_per_s"] = round(seq_rate, 3)
        log(f"[bench] serving sequential fp64 on {len(head)} requests: {seq_rate:.2f}/s")
        rate = 0.7 * seq_rate
    else:  # 0.7x the closed-loop FP64 throughput (per-stream route)
        rate = 0.7 * closed["fp64"]["solves_per_s"]
    out["open_rate_basis"] = args.open_rate
    arrivals = synth.poisson_arrivals(len(systems), rate)
    opened = {}
    for name, prec, bmax in configs:
        opened[name] = run(prec, bmax, arrivals)
        log(f"[bench] serving open-loop {name} at {rate:.2f}/s: {opened[name]}")
    out.update({"open_loop_rate_per_s": round(rate, 3), "open_loop": opened})
    return out


if __name__ == "__main__":
    main()
