"""Benchmark: time-to-1e-10 multigrid solves on one MI355X.

Default workload: 3D periodic Poisson on a uniform octree of 256^3 cells in 16^3
blocks (4096 leaf blocks), f = 32 seeded Gaussians with the mean removed, FP64, one
FMG cycle then V(2,2) cycles until the max-norm relative residual is <= 1e-10.  One
step = set the right-hand side from a device-resident array, reset phi to 0, and
solve to tolerance (the norm is checked after every cycle).

The JSON line reports leaf cell-updates per second (leaf cells x cycles / s), the
time to tolerance, the same solve in mixed precision (FP32 cycles inside FP64
iterative refinement), the HBM roofline of the finest-level smoothing kernel timed
with HIP events on the solver's stream, and the reference CPU solver timed on a
bounded sample on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_JSON = os.path.join(ROOT, "profiles", "finest_sweep_counters.json")


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=256, help="cells per axis of the benchmark grid")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-extra", action="store_true", help="skip the AMR and differentiable-solve legs")
    p.add_argument("--cpu-sample-cycles", type=int, default=1, help="V-cycles after the FMG in the CPU sample")
    p.add_argument("--workload", default="periodic256",
                   choices=["periodic256", "dirichlet2d", "amr-literal", "amr-nested", "varcoef-nested", "batch",
                            "tree-build", "paper-scaling", "convergence", "helmholtz", "divb-clean", "freespace",
                            "freespace-convergence"],
                   help="periodic256 is the benchmark line; the others print report lines")
    p.add_argument("--max-cycles", type=int, default=60)
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    return p.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: its HBM counters calibrate FETCH_SIZE /
    WRITE_SIZE, and its event-timed rate is the practical streaming bandwidth."""
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_mib": mib, "bytes_moved": 2 * n * 8, "ms": ms,
                      "gbs": 2 * n * 8 / (ms * 1e-3) / 1e9}), flush=True)


def kernel_source_hash():
    """Hash of the kernel sources (kernels, launchers and the structures they take)."""
    h = hashlib.sha256()
    for f in ("mg_kernels.hip", "mg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1901_11370_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(key, n_cells):
    """HBM bytes per launch of a finest-level smoothing kernel from committed rocprofv3
    counter runs (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration);
    None when absent, taken on other kernel sources or on another level size."""
    try:
        with open(PROFILE_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get("entries", {}).get(key)
    if d.get("source_hash") != kernel_source_hash() or not e or e.get("n_cells") != n_cells:
        return None
    return e.get("bytes_per_launch")


MAX_CYCLES = 60


def run_solve(tree, f_dev, zero_dev, tol):
    tree.set_rhs(f_dev)
    tree.set_phi(zero_dev)
    cycles, rc = tree.solve(rel_tol=tol, max_cycles=MAX_CYCLES, fmg_first=True, raise_on_fail=False)
    return cycles, rc


def timed(tree, f_dev, zero_dev, tol, steps, warmup, profile=False, fn=None):
    """W untimed steps, then exactly `steps` steps between two synchronisations; each
    step is also bracketed by HIP events on the tree's stream.  Returns (mean seconds
    per step over the region, cycles, return codes, profile record or None, per-step
    event seconds)."""
    import torch
    fn = fn or (lambda: run_solve(tree, f_dev, zero_dev, tol))
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if profile:
        tree.profile_enable(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stream = getattr(tree, "stream", None) or torch.cuda.current_stream()
    t0 = time.perf_counter()
    cyc = []
    rcs = []
    for e0, e1 in evs:
        e0.record(stream)
        c, rc = fn()
        e1.record(stream)
        cyc.append(c)
        rcs.append(rc)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    per = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    prof = tree.profile_read() if profile else None
    if profile:
        tree.profile_enable(False)
    return dt, cyc, rcs, prof, per


def _median(x):
    x = sorted(x)
    n = len(x)
    return x[n // 2] if n % 2 else 0.5 * (x[n // 2 - 1] + x[n // 2])


def cpu_info():
    """Host CPU model and the threads the reference solver's OpenMP loops use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, sample_cycles, small_n=128, tol=1e-10):
    """The reference solver, as it stands, on the host: one FMG cycle plus
    `sample_cycles` V-cycles of the benchmark workload (one thread and all threads of
    its OpenMP block loops), and the time to `tol` of the same problem at small_n^3."""
    import oracle
    from oracle import OracleTree
    from paper_1901_11370_amd import workloads as W
    d = w.domains[0]
    model, ncpu = cpu_info()
    nthreads = oracle.set_threads(0)          # the OpenMP default (OMP_NUM_THREADS)
    out = {"unit": "cell-updates/s", "kind": "oracle", "cpu_model": model, "nproc": ncpu}
    o = OracleTree(d.dim, d.base_cells, d.lo, d.hi, d.bc_kind, bs=w.bs)
    f = w.rhs(0, o.leaf_layout())
    legs = {}
    for nt in (nthreads, 1):
        oracle.set_threads(nt)
        o.set_rhs(f)
        o.set_phi(np.zeros(o.n_leaf))
        t0 = time.perf_counter()
        o.fmg()
        o.vcycle(sample_cycles)
        dt = time.perf_counter() - t0
        legs[nt] = o.n_leaf * (1 + sample_cycles) / dt
    small = W.config2(n=small_n)
    ds = small.domains[0]
    os_ = OracleTree(ds.dim, ds.base_cells, ds.lo, ds.hi, ds.bc_kind, bs=small.bs)
    fs = small.rhs(0, os_.leaf_layout())
    tt = {}
    for nt in (nthreads, 1):
        oracle.set_threads(nt)
        os_.set_rhs(fs)
        os_.set_phi(np.zeros(os_.n_leaf))
        t0 = time.perf_counter()
        hist = os_.solve(rel_tol=tol, max_cycles=40, fmg_first=True)
        tt[nt] = (time.perf_counter() - t0, len(hist), hist[-1])
    oracle.set_threads(nthreads)
    out.update({"value": legs[nthreads], "cores": nthreads, "value_1_thread": legs[1],
                "sample": f"FMG + {sample_cycles} V-cycle(s) of the same {d.base_cells[0]}^3 problem "
                          f"({o.n_leaf} leaf cells), OpenMP over the blocks of a level",
                "time_to_tol_s": {f"{small_n}^3_{nthreads}_threads": tt[nthreads][0],
                                  f"{small_n}^3_1_thread": tt[1][0]},
                "time_to_tol_cycles": tt[1][1], "time_to_tol_final_rel_residual": tt[1][2]})
    return out


def _tree_of(w, precision, mg, krylov=0, helmholtz_lambda=0.0):
    doms = [mg.Domain(d.dim, d.base_cells, d.lo, d.hi, d.bc_kind, list(d.bc_value)) for d in w.domains]
    p = mg.default_params(precision=precision, variable_eps=1 if w.variable_eps else 0, krylov=krylov,
                          helmholtz_lambda=helmholtz_lambda)
    return mg.Tree(doms, bs=w.bs, max_refine=w.max_refine, refine=w.refine, params=p)


def _inputs(w, t):
    import numpy as np
    import torch
    lay = t.leaf_layout()
    f = np.concatenate([w.rhs(i, lay[lay[:, 0] == i][:, 1:]) for i in range(len(w.domains))])
    e = None
    if w.variable_eps:
        e = torch.from_numpy(np.concatenate([w.eps(i, lay[lay[:, 0] == i][:, 1:])
                                             for i in range(len(w.domains))])).cuda()
    return torch.from_numpy(f).cuda(), e, lay


def report(a):
    """Report lines for the other workloads (not the benchmark line)."""
    import numpy as np
    import torch
    from paper_1901_11370_amd import mg
    from paper_1901_11370_amd import workloads as W

    base = {"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "data": "synthetic", "unit": "cell-updates/s",
            "higher_is_better": True}
    if a.workload == "dirichlet2d":
        w = W.config1()
        t = _tree_of(w, mg.MG_FP64, mg)
        f, _, _ = _inputs(w, t)
        z = torch.zeros_like(f)

        def ten():
            t.set_rhs(f)
            t.set_phi(z)
            t.vcycle(10)
            r, _ = t.residual_norm()
            return 10, 0
        dt, _, _, _, _ = timed(t, f, z, a.tol, a.steps, a.warmup, fn=ten)
        out = dict(base, metric="time per 10 V(2,2) cycles", value=t.n_leaf * 10 / dt, ms_per_step=dt * 1e3,
                   dtype="f64", config={"workload": "poisson2d_128^2_dirichlet_sine_10xV(2,2)", "leaf_cells": t.n_leaf},
                   final_rel_residual=t.residual_norm()[0])
        print(json.dumps(out), flush=True)
        return
    if a.workload in ("amr-literal", "amr-nested", "varcoef-nested", "helmholtz"):
        lam = 0.0
        if a.workload == "helmholtz":
            # the Helmholtz form on the benchmark grid: lambda = 100
            w, lam = W.config2(n=256), 100.0
        elif a.workload == "varcoef-nested":
            w = W.config4(nested=True)
        else:
            w = W.config3(nested=a.workload != "amr-literal")
        out = dict(base, metric="time-to-1e-10 residual", config={"workload": w.name, "helmholtz_lambda": lam})
        legs = [(mg.MG_FP64, "fp64", 0), (mg.MG_MIXED, "mixed", 0)]
        if w.variable_eps:
            # the coefficient jump stalls the plain cycles: FGMRES refinement as well
            legs.append((mg.MG_MIXED, "mixed_fgmres20", 20))
        global MAX_CYCLES
        plain_max = MAX_CYCLES
        for prec, key, kry in legs:
            # FGMRES counts every preconditioning solve as a cycle
            MAX_CYCLES = 4 * plain_max if kry else plain_max
            t = _tree_of(w, prec, mg, krylov=kry, helmholtz_lambda=lam)
            f, e, lay = _inputs(w, t)
            if e is not None:
                t.set_eps(e)
            z = torch.zeros_like(f)
            dt, cyc, rcs, _, _ = timed(t, f, z, a.tol, a.steps, a.warmup)
            r, s_ = t.solve_stats()
            out[key] = {"time_to_tol_ms": dt * 1e3, "cycles": cyc[-1], "converged": rcs[-1] == 0,
                        "final_rel_residual": float(r[-1]), "value": t.n_leaf * cyc[-1] / dt,
                        "history": [float(x) for x in r]}
            out["config"]["leaf_cells"] = t.n_leaf
            out["config"]["levels"] = t.num_levels()
            if key == "fp64":
                phi64 = t.get_phi()
            else:
                out[key]["rel_diff_vs_fp64_solution"] = float(np.abs(t.get_phi() - phi64).max() / np.abs(phi64).max())
            if kry:
                out[key]["preconditioner_applications"] = cyc[-1]
            del t
            torch.cuda.empty_cache()
        out["value"] = out["fp64"]["value"]
        out["ms_per_step"] = out["fp64"]["time_to_tol_ms"]
        out["dtype"] = "f64"
        print(json.dumps(out), flush=True)
        return
    if a.workload == "paper-scaling":
        # the paper's timing problem (Sec. 3.3): lap(phi) = 1 on the unit cube, phi = 0 on
        # the boundary, 16^3 blocks, Jacobi with 2 + 2 steps, time per V-cycle and per FMG
        # cycle averaged over 100 cycles; uniform 512^3 and 1024^3, and five levels of
        # 512^3 cells each with the refinements centred
        out = dict(base, metric="time per V-cycle and per FMG cycle (mean of 100)", unit="ms",
                   higher_is_better=False, dtype="f64",
                   config={"workload": "lap(phi)=1, phi=0 on the unit cube, 16^3 blocks, Jacobi 2+2 (weight 2/3)"})
        ncyc = 100

        def centred(levels):
            def pred(dm, lev, o, bs):
                # blocks inside the centred cube of side 2^-(lev+1) (block origin in cells)
                n = 512 << lev
                lo, hi = n // 2 - n // 2 ** (lev + 2), n // 2 + n // 2 ** (lev + 2)
                return lev < levels - 1 and all(lo <= o[q] and o[q] + bs <= hi for q in range(3))
            return pred

        cases = [("uniform_512", 512, 0, None), ("uniform_1024", 1024, 0, None),
                 ("refined_5x512", 512, 4, centred(5))]
        for name, n, mr, pred in cases:
            d = mg.Domain(3, [n] * 3, [0, 0, 0], [1, 1, 1], [mg.MG_BC_DIRICHLET] * 6)
            p = mg.default_params(smoother=mg.MG_SMOOTH_JACOBI)
            t = mg.Tree([d], bs=16, max_refine=mr, refine=pred, params=p)
            t.set_rhs(torch.ones(t.n_leaf, dtype=torch.float64, device="cuda"))
            res = {"leaf_cells": t.n_leaf, "levels": t.num_levels()}
            t.vcycle(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t.vcycle(ncyc)
            torch.cuda.synchronize()
            res["ms_per_vcycle"] = (time.perf_counter() - t0) * 1e3 / ncyc
            res["residual_after_vcycles"] = t.residual_norm()[0]
            t.set_phi(torch.zeros(t.n_leaf, dtype=torch.float64, device="cuda"))
            t.fmg(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t.fmg(ncyc)
            torch.cuda.synchronize()
            res["ms_per_fmg"] = (time.perf_counter() - t0) * 1e3 / ncyc
            res["residual_after_fmg"] = t.residual_norm()[0]
            out[name] = res
            print(name, res, file=sys.stderr, flush=True)
            del t
            torch.cuda.empty_cache()
        out["value"] = out["uniform_1024"]["ms_per_vcycle"]
        out["ms_per_step"] = out["uniform_1024"]["ms_per_vcycle"]
        print(json.dumps(out), flush=True)
        return
    if a.workload == "convergence":
        # the paper's convergence test (Sec. 3.1): residual and error per FMG iteration
        # on 64^3 cells, uniform or with two centred / corner refinement levels
        out = dict(base, metric="residual and error per FMG iteration", unit="-", dtype="f64 and mixed",
                   config={"workload": "eq. poisson-conv, 64^3 base, FMG V(2,2)"})
        for grid in ("uniform", "center", "corner"):
            w = W.x1(grid, base=64)
            for prec, key in ((mg.MG_FP64, "fp64"), (mg.MG_MIXED, "mixed")):
                t = _tree_of(w, prec, mg)
                f, _, lay = _inputs(w, t)
                d = w.domains[0]
                x = W.cell_centres(lay[:, 1:], d)
                vol = np.prod(W.cell_widths(lay[:, 1:], d), axis=1)
                sol = W.x1_solution(x)
                t.set_rhs(f)
                # boundary values of the solution at the leaf face centres, folded into f
                cells, faces = t.boundary_faces()
                t.fold_dirichlet(w.dirichlet(0, W.face_centres(lay[cells, 1:], d, faces)))
                rows = []
                for it in range(12):
                    t.fmg()
                    rm, rl = t.residual_norm()
                    e = t.get_phi() - sol
                    rows.append({"res_rel_inf": rm, "res_rel_l2": rl, "err_inf": float(np.abs(e).max()),
                                 "err_l2": float(np.sqrt(np.sum(vol * e * e)))})
                out[f"{grid}_{key}"] = {"leaf_cells": t.n_leaf, "iterations": rows}
                del t
        u, c, k = out["uniform_fp64"]["iterations"], out["center_fp64"]["iterations"], out["corner_fp64"]["iterations"]
        out["max_error_ratio_uniform_over_center"] = u[-1]["err_inf"] / c[-1]["err_inf"]
        out["l2_error_ratio_corner_over_uniform"] = k[-1]["err_l2"] / u[-1]["err_l2"]
        out["value"] = out["max_error_ratio_uniform_over_center"]
        out["ms_per_step"] = None
        print(json.dumps(out), flush=True)
        return
    if a.workload == "divb-clean":
        # elliptic divergence cleaning (Sec. 4.1) of a 256^3 periodic field (the field
        # loop of Sec. 4.2 extended along z, plus seeded non-solenoidal bumps): div B,
        # solve from phi = 0 (FMG first) to the tolerance, projection with the energy fix
        import torch
        w = W.divb_periodic(a.n)
        d = w.domains[0]
        out = dict(base, metric="divergence cleaning time", dtype="f64 and mixed",
                   config={"workload": f"divb_clean_periodic3d_{a.n}^3_fieldloop+bumps_to_{a.tol:g}"})
        for prec, key in ((mg.MG_FP64, "fp64"), (mg.MG_MIXED, "mixed")):
            t = _tree_of(w, prec, mg)
            lay = t.leaf_layout()
            B0 = torch.from_numpy(W.field_loop_B(d, W.cell_centres(lay[:, 1:], d))).cuda()
            e0 = (1.0 + 0.5 * (B0 * B0).sum(0)).contiguous()
            B, e = B0.clone(), e0.clone()
            z = torch.zeros(t.n_leaf, dtype=torch.float64, device="cuda")
            for order in (2, 4):
                def clean():
                    B.copy_(B0)
                    e.copy_(e0)
                    t.divb_rhs(B, order)
                    t.set_phi(z)
                    c, rc = t.solve(rel_tol=a.tol, max_cycles=MAX_CYCLES, fmg_first=True, raise_on_fail=False)
                    t.divb_project(B, e)
                    return c, rc

                dt, cyc, rcs, _, _ = timed(t, None, None, a.tol, a.steps, a.warmup, fn=clean)

                def part(fn):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(a.steps):
                        fn()
                    torch.cuda.synchronize()
                    return (time.perf_counter() - t0) / a.steps * 1e3

                res = {"ms_per_clean": dt * 1e3, "cycles": cyc[-1], "converged": all(rc == 0 for rc in rcs),
                       "ms_divb_rhs": part(lambda: t.divb_rhs(B0, order)),
                       "ms_project": part(lambda: t.divb_project(B, e)),
                       "leaf_cells": t.n_leaf}
                res["cells_per_s"] = t.n_leaf / dt
                out[f"{key}_order{order}"] = res
            del t
        out["value"] = out["fp64_order4"]["cells_per_s"]
        out["ms_per_step"] = out["fp64_order4"]["ms_per_clean"]
        out["note"] = "ms_per_clean includes restoring B and e from a copy (about 0.15 ms)"
        print(json.dumps(out), flush=True)
        return
    if a.workload == "freespace":
        # free-space boundaries (Sec. 2.8) on the paper's test (Sec. 3.2: Gaussian source,
        # sigma 0.1, unit cube centred at the origin), 256^3 leaf cells: boundary values
        # from the charges 2^k coarser, folded into f, then FMG + V-cycles to the tolerance
        w = W.freespace_gauss((a.n,))
        out = dict(base, metric="free-space boundary values + solve time", dtype="f64 and mixed",
                   config={"workload": f"freespace_gauss_{a.n}^3_sigma0.1_to_{a.tol:g}"})
        for k in (2, 1):
            for prec, key in ((mg.MG_FP64, "fp64"), (mg.MG_MIXED, "mixed")):
                t = _tree_of(w, prec, mg)
                lay = t.leaf_layout()
                f = torch.from_numpy(w.rhs(0, lay[:, 1:])).cuda()

                def bc():
                    t.set_rhs(f)
                    t.freespace_bc(k)

                def run():
                    t.set_rhs(f)
                    t.freespace_guess(k)   # phi: the far-field guess
                    t.freespace_bc(k)
                    return t.solve(rel_tol=a.tol, max_cycles=MAX_CYCLES, fmg_first=True, raise_on_fail=False)

                dt, cyc, rcs, _, _ = timed(t, None, None, a.tol, a.steps, a.warmup, fn=run)
                for _ in range(a.warmup):
                    bc()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(a.steps):
                    bc()
                torch.cuda.synchronize()
                ms_bc = (time.perf_counter() - t0) / a.steps * 1e3
                e = t.get_phi() - w.target(0, lay[:, 1:])
                nc = a.n >> k
                pairs = 6 * (nc + 2) ** 2 * nc ** 3
                res = {"ms_total": dt * 1e3, "ms_boundary_values": ms_bc, "cycles": cyc[-1],
                       "converged": all(rc == 0 for rc in rcs), "coarse_cells": nc ** 3,
                       "plane_points": 6 * (nc + 2) ** 2, "pair_terms_per_s": pairs / (ms_bc * 1e-3),
                       "err_l2": float(np.sqrt(np.mean(e * e))), "err_max": float(np.max(np.abs(e)))}
                out[f"{key}_coarsen{k}"] = res
                del t
        out["value"] = a.n ** 3 / (out["fp64_coarsen2"]["ms_total"] * 1e-3)
        out["ms_per_step"] = out["fp64_coarsen2"]["ms_total"]
        out["note"] = ("ms_boundary_values includes setting f (a device copy); pair terms: plane points x "
                       "coarse cells of the direct Green's-function sum")
        print(json.dumps(out), flush=True)
        return
    if a.workload == "freespace-convergence":
        # the paper's Fig. free-space-error (Sec. 3.2): error of the solution after two FMG
        # cycles against eq. gauss-sol versus grid size, with the free-space values taken
        # one and two levels below the finest (charges 2x and 4x coarser)
        out = dict(base, metric="free-space test: error after two FMG cycles and at the tolerance", unit="L2 error",
                   higher_is_better=False, dtype="f64",
                   config={"workload": "freespace_gauss_sigma0.1_fmg2_64-512"})
        rows = []
        for n in (64, 128, 256, 512):
            w = W.freespace_gauss((n,))
            lay = None
            for k in (1, 2):
                t = _tree_of(w, mg.MG_FP64, mg)
                if lay is None:
                    lay = t.leaf_layout()
                    f = torch.from_numpy(w.rhs(0, lay[:, 1:])).cuda()
                    exact = w.target(0, lay[:, 1:])
                t.set_rhs(f)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t.freespace_bc(k)
                torch.cuda.synchronize()
                ms_bc = (time.perf_counter() - t0) * 1e3
                t.set_phi(torch.zeros_like(f))
                t.fmg(2)
                e = t.get_phi() - exact
                ex = np.abs(exact).max()
                row = {"n": n, "levels_below": k, "fmg2_err_l2": float(np.sqrt(np.mean(e * e))),
                       "fmg2_err_max_rel": float(np.max(np.abs(e)) / ex), "ms_boundary_values": ms_bc}
                # the same two FMG cycles from the far-field guess
                t2 = _tree_of(w, mg.MG_FP64, mg)
                t2.set_rhs(f)
                t2.freespace_guess(k)
                t2.freespace_bc(k)
                t2.fmg(2)
                e2 = t2.get_phi() - exact
                row.update({"guess_fmg2_err_l2": float(np.sqrt(np.mean(e2 * e2))),
                            "guess_fmg2_err_max_rel": float(np.max(np.abs(e2)) / ex)})
                del t2, e2
                # then V-cycles to the tolerance: the discretisation error itself
                c, rc = t.solve(rel_tol=a.tol, max_cycles=MAX_CYCLES, fmg_first=False, raise_on_fail=False)
                e = t.get_phi() - exact
                row.update({"cycles_after": c, "err_l2": float(np.sqrt(np.mean(e * e))),
                            "err_max_rel": float(np.max(np.abs(e)) / ex)})
                rows.append(row)
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
                del t, e
        out["rows"] = rows
        out["value"] = rows[-1]["err_l2"]
        out["ms_per_step"] = None
        print(json.dumps(out), flush=True)
        return
    if a.workload == "tree-build":
        # step a1: host construction of the tree and tables (the paper quotes ~0.3 s for
        # a uniform 1024^3 grid of 16^3 blocks), then binding (table upload, field init)
        out = dict(base, metric="tree build time", unit="s", higher_is_better=False, dtype="-",
                   config={"workload": "uniform 1024^3 in 16^3 blocks, and the nested AMR tree"})
        d = mg.Domain(3, [1024] * 3, [0, 0, 0], [1, 1, 1], [mg.MG_BC_DIRICHLET] * 6)
        times = []
        for _ in range(max(a.steps, 1)):
            t0 = time.perf_counter()
            t = mg.Tree([d], bs=16, bind=False)
            times.append(time.perf_counter() - t0)
            del t
        out["create_s_1024"] = sorted(times)[len(times) // 2]
        t = mg.Tree([d], bs=16, bind=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.bind()                      # store allocation, table upload, field initialisation
        torch.cuda.synchronize()
        out["bind_s_1024"] = time.perf_counter() - t0
        out["store_gb_1024"] = t.storage_bytes / 1e9
        del t
        torch.cuda.empty_cache()
        w = W.config3(nested=True)
        dd = w.domains[0]
        t0 = time.perf_counter()
        t = mg.Tree([mg.Domain(dd.dim, dd.base_cells, dd.lo, dd.hi, dd.bc_kind)], bs=16, max_refine=w.max_refine,
                    refine=w.refine, bind=False)
        out["create_s_nested_amr"] = time.perf_counter() - t0
        out["value"] = out["create_s_1024"]
        out["ms_per_step"] = out["create_s_1024"] * 1e3
        print(json.dumps(out), flush=True)
        return
    if a.workload == "batch":
        from paper_1901_11370_amd.autograd import mg_solve
        w = W.config5()
        t = _tree_of(w, mg.MG_MIXED, mg)
        f, e, lay = _inputs(w, t)
        tgt = torch.from_numpy(np.concatenate([w.target(i, lay[lay[:, 0] == i][:, 1:])
                                               for i in range(len(w.domains))])).cuda()

        def fwd_bwd():
            ff = f.clone().requires_grad_(True)
            ee = e.clone().requires_grad_(True)
            phi = mg_solve(ff, ee, t, a.tol, a.max_cycles)
            J = 0.5 * torch.sum((phi - tgt) ** 2)
            J.backward()
            return 1, 0
        t.set_eps(e)
        t.set_rhs(f)
        t.set_phi(torch.zeros_like(f))
        t0 = time.perf_counter()
        cyc, _ = t.solve(rel_tol=a.tol, max_cycles=a.max_cycles, raise_on_fail=False)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        fwd_res = [float(x) for x in t.domain_residual_norms()[0]]
        dt, _, _, _, _ = timed(t, f, None, a.tol, a.steps, a.warmup, fn=fwd_bwd)
        out = dict(base, metric="forward + adjoint backward time", value=t.n_leaf / dt, ms_per_step=dt * 1e3,
                   dtype="f32 cycles in f64 refinement",
                   config={"workload": w.name, "leaf_cells": t.n_leaf, "domains": len(w.domains)},
                   forward_ir_steps=cyc, forward_ms=t_fwd * 1e3, forward_domain_residuals=fwd_res)
        print(json.dumps(out), flush=True)
        return


def roofline_of(prof, kernel, dtp, key=None, n_cells=None):
    """Roofline record of the event-timed finest-level smoothing launches; `traffic` from
    the counter runs stored under `key` for a finest level of n_cells cells."""
    launches, total_ms, bytes_per = prof
    if not launches:
        return None
    avg_ms = total_ms / launches
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": kernel, "avg_us": avg_ms * 1e3, "launches": launches,
            "algorithmic_bytes_per_launch": bytes_per, "events_region_ms_per_step": dtp * 1e3,
            "traffic": traffic_from_profile(key, n_cells) if key else None}


def _finest_cells(t):
    """Cells of the tree's finest level (the level whose sweeps the roofline times)."""
    _, ncell = t.level_blocks()
    return int(ncell[-1])


def amr_leg(a, mg, W):
    """The AMR workload at its ~1e8-leaf-cell layout (base 128^3, three refinement levels
    nested around the centre, four Gaussian sources, phi = 0 on the boundary): FP64 and
    mixed time to tolerance, with the event-timed finest-level smoothing kernel."""
    import torch
    w = W.config3(nested=True)
    steps = max(1, min(a.steps, 8))
    out = {"workload": "amr3d_base128_3levels_nested_4gauss_dirichlet_fmg+V(2,2)_to_1e-10"}
    for prec, key in ((mg.MG_FP64, "fp64"), (mg.MG_MIXED, "mixed")):
        t = _tree_of(w, prec, mg)
        f, _, _ = _inputs(w, t)
        z = torch.zeros_like(f)
        dt, cyc, rcs, _, per = timed(t, f, z, a.tol, steps, 2)
        r, _ = t.solve_stats()
        dtp, _, _, prof, _ = timed(t, f, z, a.tol, 2, 1, profile=True)
        leg = {"time_to_tol_ms": dt * 1e3, "time_to_tol_ms_median_events": _median(per) * 1e3,
               "cycles": cyc[-1], "converged": all(rc == 0 for rc in rcs), "final_rel_residual": float(r[-1]),
               "leaf_cell_cycles_per_s": t.n_leaf * cyc[-1] / dt, "leaf_cells": t.n_leaf,
               "roofline": roofline_of(prof, f"k_gsrb<{'double' if prec == 0 else 'float'},3,16> finest AMR level "
                                             "(one colour)", dtp, f"amr_nested_{key}", _finest_cells(t))}
        if key == "fp64":
            phi64 = t.get_phi()
        else:
            leg["rel_diff_vs_fp64_solution"] = float(np.abs(t.get_phi() - phi64).max() / np.abs(phi64).max())
        out[key] = leg
        del t, f, z
        torch.cuda.empty_cache()
    return out


def batch_leg(a, mg, W):
    """The differentiable solve: forward (FP32 cycles in FP64 refinement to the
    tolerance) and adjoint backward of the six-member batch (64^3 ... 256^3, log-normal
    eps), with the event-timed finest-level variable-coefficient FP32 sweep."""
    import torch
    from paper_1901_11370_amd.autograd import mg_solve
    w = W.config5()
    t = _tree_of(w, mg.MG_MIXED, mg)
    f, e, lay = _inputs(w, t)
    tgt = torch.from_numpy(np.concatenate([w.target(i, lay[lay[:, 0] == i][:, 1:])
                                           for i in range(len(w.domains))])).cuda()

    def fwd_bwd():
        ff = f.clone().requires_grad_(True)
        ee = e.clone().requires_grad_(True)
        phi = mg_solve(ff, ee, t, a.tol, a.max_cycles)
        J = 0.5 * torch.sum((phi - tgt) ** 2)
        J.backward()
        return 1, 0
    steps = max(1, min(a.steps, 8))
    dt, _, _, _, per = timed(t, f, None, a.tol, steps, 2, fn=fwd_bwd)
    t.set_eps(e)

    def fwd():
        t.set_rhs(f)
        t.set_phi(torch.zeros_like(f))
        return t.solve(rel_tol=a.tol, max_cycles=a.max_cycles, raise_on_fail=False)
    dtf, cyc, rcs, _, _ = timed(t, f, None, a.tol, steps, 1, fn=fwd)
    dtp, _, _, prof, _ = timed(t, f, None, a.tol, 2, 1, profile=True, fn=fwd)
    out = {"workload": "diffsolve3d_batch6 (64^3..256^3, log-normal eps), J = 1/2 |phi - phi_t|^2",
           "leaf_cells": t.n_leaf, "fwd_bwd_ms": dt * 1e3, "fwd_bwd_ms_median_events": _median(per) * 1e3,
           "forward_ms": dtf * 1e3, "forward_ir_steps": cyc[-1], "forward_converged": all(rc == 0 for rc in rcs),
           "roofline": roofline_of(prof, "k_gsrb<float,3,16,var-eps> finest level (one colour)", dtp,
                                   "diffsolve_batch_fp32", _finest_cells(t))}
    del t
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(mib=1024):
    """Event-timed device-to-device copy of `mib` MiB: the practical streaming rate."""
    import torch
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def main():
    a = _args()
    global MAX_CYCLES
    MAX_CYCLES = a.max_cycles
    if a.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU; --gpus {a.gpus} is not supported "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.workload != "periodic256":
        report(a)
        return
    import torch
    from paper_1901_11370_amd import mg
    from paper_1901_11370_amd import workloads as W

    w = W.config2(n=a.n)
    d = w.domains[0]
    dom = mg.Domain(d.dim, d.base_cells, d.lo, d.hi, d.bc_kind)
    t64 = mg.Tree([dom], bs=16, params=mg.default_params(precision=mg.MG_FP64))
    lay = t64.leaf_layout()
    f = w.rhs(0, lay[:, 1:])
    f_dev = torch.from_numpy(f).to("cuda")
    zero_dev = torch.zeros_like(f_dev)
    nb, ncell = t64.level_blocks()
    n_leaf = t64.n_leaf

    # headline timed region: cycle sequences replayed from captured graphs
    dt, cyc, rcs, _, per = timed(t64, f_dev, zero_dev, a.tol, a.steps, a.warmup)
    res, secs = t64.solve_stats()
    # roofline: HIP events around every finest-level smoothing launch over a second
    # timed region of the same solves (events need the kernels launched one by one)
    dtp, _, _, prof, _ = timed(t64, f_dev, zero_dev, a.tol, a.steps, 1, profile=True)
    cycles = cyc[-1]
    # smoothing updates per cycle: every level's cells, (n_down + n_up) sweeps
    gs_updates = float(ncell.sum()) * 4 * cycles
    out = {
        "metric": "cell-updates/s & time-to-1e-10 residual, FP64 vs mixed; % peak HBM",
        "value": n_leaf * cycles / dt,
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"poisson3d_{a.n}^3_periodic_32gauss_fmg+V(2,2)_to_{a.tol:g}",
                   "leaf_cells": n_leaf, "block": "16^3", "levels": int(len(nb))},
        "time_to_tol_ms": dt * 1e3,
        "time_to_tol_ms_median_events": _median(per) * 1e3,
        "cycles_to_tol": cycles,
        "converged": all(rc == 0 for rc in rcs),
        "final_rel_residual": float(res[-1]),
        "gs_point_updates_per_s": gs_updates / dt,
    }
    roof = roofline_of(prof, "k_gsrb<double,3,16> finest level (one colour)", dtp, "poisson3d_256_fp64",
                       int(ncell[-1]))
    if roof:
        roof["copy_gbs_in_run"] = copy_bandwidth()
        roof["frac_of_copy"] = roof["achieved"] / roof["copy_gbs_in_run"]
        out["roofline"] = roof

    if not a.no_mixed:
        tmx = mg.Tree([dom], bs=16, params=mg.default_params(precision=mg.MG_MIXED))
        dtm, cycm, rcsm, _, perm = timed(tmx, f_dev, zero_dev, a.tol, a.steps, a.warmup)
        resm, _ = tmx.solve_stats()
        dtmp, _, _, profm, _ = timed(tmx, f_dev, zero_dev, a.tol, 2, 1, profile=True)
        phi64 = t64.get_phi()
        phim = tmx.get_phi()
        p64 = phi64 - phi64.mean()
        pm = phim - phim.mean()
        out["mixed"] = {"time_to_tol_ms": dtm * 1e3, "time_to_tol_ms_median_events": _median(perm) * 1e3,
                        "ir_steps": cycm[-1], "converged": all(rc == 0 for rc in rcsm),
                        "final_rel_residual": float(resm[-1]),
                        "value": n_leaf * cycm[-1] / dtm, "unit": "cell-updates/s",
                        "speedup_vs_fp64": dt / dtm,
                        "rel_diff_vs_fp64_solution": float(np.abs(pm - p64).max() / np.abs(p64).max()),
                        "roofline": roofline_of(profm, "k_gsrb<float,3,16> finest level (one colour)", dtmp,
                                                "poisson3d_256_fp32", int(ncell[-1]))}
        del tmx
    del t64
    torch.cuda.empty_cache()
    if not a.no_extra:
        out["amr_nested"] = amr_leg(a, mg, W)
        out["diffsolve_batch"] = batch_leg(a, mg, W)

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_sample_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
