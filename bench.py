"""Benchmark: shift-and-invert QEP eigenpairs/s on one MI355X, rIGA vs IGA.

Workload: scalar damped-wave QEP (lam^2 M + lam C + K) u = 0 on the unit
square, p = 3 B-splines on 256 x 256 elements, homogeneous Dirichlet,
Rayleigh damping C = 0.05 M + 0.005 K, the 40 eigenpairs nearest sigma = 2
with a Krylov subspace of 80.  rIGA places C^0 hyperplanes every 16 elements
(82,369 dofs); IGA is the maximum-continuity space (66,049 dofs).

One step = the whole hot path for the rIGA discretisation: assemble K, M, C;
factor Q(sigma); Krylov-Schur eigensolve with the FB solves; eigenvector
normalisation and residuals.  Inputs are generated (and resident on the
device) before the timed region.  The IGA discretisation and the CPU oracle are
measured after the timed steps and reported beside it.

The precision form (FP32 fronts + FP64 refinement against the FP64 path on
the p=4, 1024^2, s=32 workload) and the batching form (256 uneven problems
solved together) are measured last and reported beside it.

The undamped case (C = 0: all eigenvalues of K u = mu M u in an interval by
spectrum slicing) on the same mesh, rIGA and IGA, is reported last, and the
headline step with the Krylov basis in compact two-level (TOAR) form beside
the full basis, and the headline mesh with a gyroscopic (skew) part in the
damping, factored by LU.  The curl-conforming vector space (p=3, 256^2, perfect
conductor) closes the run: factorization, FB elimination and Maxwell spectrum
slicing, rIGA against IGA, and its conductive QEP at the complex target 7i
(the real part of the shift-and-invert operator); the vibroacoustic cavity on
the divergence-conforming space (absorbing top wall) at 0.5 + 7i.  `--flop-table` prints the host-side symbolic cost
ratios of that space for p = 3..6 (the quantities of tab:FlopTest) and exits;
`--flop-test` runs that space's conductive QEP at the target 7i for p = 3..5 on
the device (100 pairs) and prints the same ratios from the runs' counts and times.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-iga] [--no-mixed] [--no-batch]
                       [--no-undamped] [--no-toar] [--no-gyro] [--no-hcurl] [--no-em] [--no-vibro]
                       [--basis full|toar]
                       [--flop-table] [--flop-test]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s + factor GFLOP/s, rIGA vs IGA, FP64 vs mixed @1e-10 eig err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def run_config(torch, riga, P, steps, warmup, block, flags=0):
    pr = riga.Problem(P.p, P.ne, P.hyper_every)
    info = pr.info

    def one():
        pr.assemble(P.alpha, P.beta)
        pr.factor(P.sigma)
        return pr.eigs(P.nev, P.m, block=block, seed=0, vectors=True, flags=flags)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for _ in range(steps):
        outs.append(one())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lam, X, eta, nconv, st = outs[-1]
    good = int(sum(1 for e in eta[:nconv] if e <= 1e-10))
    stats = pr.stats()
    ms = (t1 - t0) * 1e3 / max(steps, 1)
    res = {
        "ndof": int(info["ndof"]), "nnz": int(info["nnz"]), "tree_levels": int(info["height"]),
        "leaves": int(info["nleaves"]), "max_front": int(info["max_front"]),
        "factor_entries": int(info["factor_entries"]),
        "ms_per_step": ms,
        "eigenpairs_per_s": good * 1e3 / ms,
        "pairs_ok": good, "status": int(st),
        "factor_ms": stats["t_factor_ms"], "eigs_ms": stats["t_eigs_ms"], "eigs_host_ms": stats["t_host_ms"],
        # algorithmic flops: the symbolic count sum_j (c_j^2 + 2 c_j) of the elimination order used
        "factor_gflops": info["factor_flops"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
        "factor_gflop_algorithmic": info["factor_flops"] / 1e9,
        "factor_gflops_dense": info["factor_flops_dense"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
        "factor_gflop_dense": info["factor_flops_dense"] / 1e9,
        "solve_factor_mb": info["solve_bytes"] / 1e6,
        "n_it": int(stats["n_it"]), "n_fb": int(stats["n_fb"]), "n_mv": int(stats["n_mv"]),
        "n_vv": int(stats["n_vv"]),
        "max_eta": float(max(eta)),
    }
    return pr, res, lam


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_sweeps_p3_256x256_s16.json")


def measured_traffic(kernel, block):
    """HBM bytes per launch of a sweep kernel from the committed counter record
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when a source the
    traffic depends on (sweep kernels, task layout, elimination tree) has
    changed since the counters were taken or the launch shape differs."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_RECORD))
        for src, want in rec["source_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != want:
                return None
    except (OSError, ValueError, KeyError, AttributeError):
        return None
    if block != 2:
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def roofline(pr, res, block):
    """Roofline of the kernel family with the most time in one step, timed live
    with HIP events on the solver's stream (average duration of one launch)."""
    fam = {}
    for which, name in ((0, "k_fwd"), (1, "k_bwd"), (2, "k_front_factor")):
        reps = 3 if which == 2 else 30
        ms, work, levels = pr.time_kernel(which, nrhs=block, reps=reps)
        # launches per step: one per level per forward/backward sweep, one per level per factorization
        per_step = levels * (res["n_fb"] // block + 1) if which < 2 else levels
        fam[name] = (ms, work, per_step * ms)
    name = max(fam, key=lambda k: fam[k][2])
    ms, work, _ = fam[name]
    if name == "k_front_factor":
        achieved = work / (ms * 1e-3) / 1e12
        out = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
               "frac": achieved / FP64_PEAK_TFS}
    else:
        achieved = work / (ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": achieved / HBM_PEAK_GBS}
    out.update({"traffic": measured_traffic(name, block), "kernel": name, "avg_launch_us": ms * 1e3,
                "work_per_launch": work,
                "step_ms_by_kernel": {k: v[2] for k, v in fam.items()},
                # factor bytes one forward + backward solve reads: below the chip's 256 MB
                # last-level cache (MALL), so the sweeps of this workload can hit it
                "solve_factor_mb": res["solve_factor_mb"], "mall_resident": res["solve_factor_mb"] < 256.0})
    return out


def gyroscopic_form(torch, riga, W, steps, block):
    """The headline mesh (rIGA and IGA) with a skew-symmetric part in the
    damping: LU factorisation of the nonsymmetric Q(sigma) and the eigensolve,
    timed like the headline step (assemble + factor + eigs per step)."""
    import numpy as np

    out, lams = {}, {}
    for s in (16, 0):
        P = W.cfg_gyro(s)
        pr = riga.Problem(P.p, P.ne, P.hyper_every)
        info = pr.info

        def one():
            pr.assemble(P.alpha, P.beta, gyro=P.extra["gyro"])
            pr.factor(P.sigma)
            return pr.eigs(P.nev, P.m, block=block, seed=0, vectors=True)

        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lam, X, eta, nconv, st = one()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        stats = pr.stats()
        good = int(sum(1 for e in eta[:nconv] if e <= 1e-10))
        out["riga" if s else "iga"] = {
            "workload": f"p={P.p}, {P.ne}x{P.ne}, " + (f"rIGA s={s}" if s else "IGA") +
                        f", C = {P.alpha}M + {P.beta}K + G(g={P.extra['gyro']}), {P.nev} pairs nearest "
                        f"sigma={P.sigma}, subspace {P.m}",
            "ndof": int(info["ndof"]), "ms_per_step": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
            "status": int(st), "factor_ms": stats["t_factor_ms"], "eigs_ms": stats["t_eigs_ms"],
            # an LU without pivoting does twice the work of the Cholesky of the same pattern
            "factor_gflops_algorithmic": 2.0 * info["factor_flops"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
            "n_it": int(stats["n_it"]), "n_fb": int(stats["n_fb"]), "max_eta": float(max(eta)),
            "max_abs_re_over_abs": float(np.max(np.abs(np.real(lam)) / np.abs(lam))),
        }
        lams["riga" if s else "iga"] = (P, lam)
        pr.close()
    return out, lams


def oracle_check_gyro(lams):
    """Eigenvalues of the gyroscopic leg against the oracle's 1-D y-mode
    closed form: part of the CPU-baseline leg."""
    import numpy as np

    from oracle import gyro as ogyro

    res = {}
    for k, (P, lam) in lams.items():
        ref = ogyro.gyro_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.extra["gyro"][0], P.sigma, P.nev)
        rel = np.abs(np.asarray(lam) - ref) / np.abs(ref)
        res[k] = (float(rel.max()), int((rel <= 1e-10).sum()))
    return res


def compact_basis_form(torch, riga, W, steps, block):
    """The headline workload (rIGA and IGA) with the Krylov basis in compact
    two-level form (RIGA_EIGS_TOAR): the same step, timed the same way, and
    the N-long Krylov storage of both forms."""
    out, lams = {}, {}
    for s in (16, 0):
        P = W.cfg_riga_vs_iga(s)
        pr, res, lam = run_config(torch, riga, P, steps, 1, block, flags=riga.RIGA_EIGS_TOAR)
        ldh = P.m + 2 * block
        res["krylov_storage_mb"] = 2 * res["ndof"] * ldh * 8 / 1e6          # U and its restart copy
        res["full_basis_storage_mb"] = 6 * res["ndof"] * ldh * 8 / 1e6       # V_u, V_l, M V_l and copies
        res["toar_drop"] = pr.stats()["toar_drop"]
        out["riga" if s else "iga"] = res
        lams["riga" if s else "iga"] = (P, lam)
        pr.close()
    return out, lams


def precision_form(torch, riga, W, ir_tol=1e-9):
    """FP64 path vs the mixed path (FP32 fronts below the FP64 root level, FP64
    refinement of every solve) on the p=4, 1024^2, s=32 workload with a
    lognormal element damping field: phase times, eigenpairs/s and the error of
    every mixed eigenvalue against the FP64 one."""
    import numpy as np

    P = W.cfg_precision()
    pr = riga.Problem(P.p, P.ne, P.hyper_every)
    info = pr.info
    c = torch.from_numpy(P.c_elem).to(pr.device)
    out = {"workload": f"p={P.p}, {P.ne}x{P.ne}, s={P.hyper_every}, c_e lognormal(-3,0.5) seed 0, "
                       f"sigma={P.sigma}, {P.nev} pairs, subspace {P.m}", "ndof": int(info["ndof"])}
    lams = {}
    for prec in ("fp64", "mixed"):
        def one():
            pr.assemble(0.0, 0.0, c)
            if prec == "fp64":
                pr.factor(P.sigma)
                hist = None
            else:
                hist = pr.factor(P.sigma, "mixed", fp64_levels=1, ir_sweeps=-1, ir_tol=ir_tol)
            r = pr.eigs(P.nev, P.m, block=2, seed=0, vectors=False)
            return hist, r
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, (lam, _, eta, nconv, st) = one()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        stats = pr.stats()
        good = int(sum(1 for e in eta[:nconv] if e <= 1e-10))
        lams[prec] = lam
        sweeps = {}
        for which, name in ((0, "k_fwd"), (1, "k_bwd")):
            kms, work, levels = pr.time_kernel(which, nrhs=2, reps=10)
            # the factor of this workload (2.2 GB in FP64) streams from HBM on every sweep
            sweeps[name] = {"avg_launch_us": kms * 1e3, "levels": levels, "work_per_launch": work,
                            "achieved_gbs": work / (kms * 1e-3) / 1e9,
                            "frac": work / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        rec = {"ms_per_step": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
               "factor_ms": stats["t_factor_ms"], "eigs_ms": stats["t_eigs_ms"],
               "factor_gflops": info["factor_flops"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
               "factor_gflops_dense": info["factor_flops_dense"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
               "n_fb": int(stats["n_fb"]), "n_ir": int(stats["n_ir"]), "max_eta": float(max(eta)),
               "sweep_roofline": sweeps}
        if hist is not None:
            rec["ir_sweeps"] = pr.ir_sweeps()
            rec["ir_tol"] = ir_tol
            rec["ir_residual_history"] = [float(x) for x in hist]
        out[prec] = rec
    rel = np.abs(lams["mixed"] - lams["fp64"]) / np.abs(lams["fp64"])
    out["mixed"]["rel_err_vs_fp64"] = [float(x) for x in rel]
    out["mixed"]["max_rel_err_vs_fp64"] = float(rel.max())
    pr.close()
    return out


def batching_form(torch, riga, W, steps=2):
    """The batching workload: 256 independent problems (ne in {32..128}, p in
    {2,3,4}, s=8, seeded damping and shifts, 8 pairs each) assembled, factored
    and solved together; sweep shapes autotuned on the forest first.  The
    single-problem path on the first 32 problems is timed beside it."""
    probs = W.cfg_batch()
    B = riga.Batch([(P.p, P.ne, P.hyper_every) for P in probs])
    al, be, sg = [P.alpha for P in probs], [P.beta for P in probs], [P.sigma for P in probs]
    B.assemble(al, be)
    B.factor(sg)
    before, after = B.autotune(2, 5)

    def one():
        B.assemble(al, be)
        B.factor(sg)
        return B.eigs(8, 20, block=2, seed=0)

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lam, _, eta, nconv, st = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    s = B.stats()
    good = int(sum(int(((eta[i][:nconv[i]]) <= 1e-10).sum()) for i in range(len(probs))))
    out = {"workload": "256 problems, ne in {32,48,64,96,128}, p in {2,3,4}, s=8, Rayleigh alpha~U[0,0.2], "
                       "beta~U[0,0.02], sigma~U[0.5,4] (seed 1), 8 pairs each, subspace 20",
           "total_dofs": int(B.total), "ms_per_step": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
           "assemble_ms": s["t_assemble_ms"], "factor_ms": s["t_factor_ms"], "eigs_ms": s["t_eigs_ms"],
           "eigs_host_ms": s["t_host_ms"],
           "lockstep_cycles": int(s["n_it"]), "resolved_one_by_one": int(s["n_resolved"]),
           "max_eta": float(eta.max()), "autotune_forest_solve_ms": {"before": before, "after": after}}
    B.close()
    # the single-problem path, one problem after another
    t0 = time.perf_counter()
    cnt = 0
    for P in probs[:32]:
        pr = riga.Problem(P.p, P.ne, P.hyper_every)
        pr.assemble(P.alpha, P.beta)
        pr.factor(P.sigma)
        _, _, e1, n1, _ = pr.eigs(8, 20, block=2, seed=0, vectors=False)
        cnt += int((e1[:n1] <= 1e-10).sum())
        pr.close()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["one_by_one_first32_eigenpairs_per_s"] = cnt / t
    return out


def oracle_check(P, lam_gpu):
    """Relative error of every returned eigenvalue against the oracle's closed
    form (Rayleigh damping: the 1-D pencil's Kronecker sums, seconds on the
    host) and the number within 1e-10: part of the CPU-baseline leg."""
    import numpy as np

    from oracle import eigen as oeig

    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    rel = np.abs(np.asarray(lam_gpu)[:len(ref)] - ref) / np.abs(ref)
    return float(rel.max()), int((rel <= 1e-10).sum())


def undamped_form(torch, riga, W):
    """The undamped case (C = 0) on the headline mesh, rIGA and IGA: every
    eigenvalue of K u = mu M u in [0, 1500) by spectrum slicing (inertia of
    signed factorizations, block Lanczos per slice), one warm-up and one timed
    call each; eigenpairs/s counts the returned pairs with scaled residual
    <= 1e-10."""
    out, mus = {}, {}
    for s in (16, 0):
        P = W.cfg_undamped(s)
        a, b = P.extra["interval"]
        pr = riga.Problem(P.p, P.ne, P.hyper_every)
        pr.assemble(0.0, 0.0)
        pr.gep_slice(a, b, max_slice=P.extra["max_slice"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, U, eta, count, st, stats = pr.gep_slice(a, b, max_slice=P.extra["max_slice"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        good = int(sum(1 for e in eta if e <= 1e-10))
        st_h = pr.stats()
        out["riga" if s else "iga"] = {
            "workload": f"p={P.p}, {P.ne}x{P.ne}, " + (f"rIGA s={s}" if s else "IGA") +
                        f", all mu in [{a:g}, {b:g}), slices of <= {P.extra['max_slice']}",
            "ndof": int(pr.ndof), "count": int(count), "found": int(len(mu)), "status": int(st),
            "ms": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
            "factor_ms_total": st_h["t_factor_ms"], "max_eta": float(max(eta)) if len(eta) else None,
            **stats}
        mus["riga" if s else "iga"] = (P, mu)
        pr.close()
    return out, mus


def oracle_check_undamped(mus):
    """Count and eigenvalues of the undamped leg against the oracle's closed
    form (Kronecker sums of the 1-D pencil): part of the CPU-baseline leg."""
    import numpy as np

    from oracle import gep as ogep

    res = {}
    for k, (P, mu) in mus.items():
        a, b = P.extra["interval"]
        ref = ogep.gep_closed(P.p, P.ne, P.hyper_every, a, b)
        rel = float(np.max(np.abs(mu - ref) / np.abs(ref))) if len(ref) == len(mu) and len(mu) else None
        res[k] = (len(ref), rel)
    return res


def vector_space_form(torch, riga, W, reps=10):
    """The curl-conforming space (p=3, 256x256, perfect conductor), rIGA and
    IGA: the conductive form C = 0.05 M + 0.005 K factored at sigma=2 (one
    warm-up and one timed factorization; GFLOP/s from the symbolic count of
    the elimination order used), the solve of two right-hand sides (FB
    elimination, mean of `reps`), and the Maxwell form K u = mu M u with
    every eigenvalue in [1, 150) by spectrum slicing.  The cost ratios IGA /
    rIGA are the quantities of tab:FlopTest measured on the device."""
    out, mus = {}, {}
    for s in (16, 0):
        P = W.cfg_hcurl(s)
        space = P.extra["space"]
        a, b = P.extra["interval"]
        pr = riga.Problem(P.p, P.ne, P.hyper_every, space=space)
        info = pr.info
        pr.assemble(P.alpha, P.beta)
        pr.factor(P.sigma)
        pr.factor(P.sigma)
        t_fac = pr.stats()["t_factor_ms"]
        rhs = torch.randn((2, pr.ndof), dtype=torch.float64, device="cuda")
        pr.solve_q(rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pr.solve_q(rhs)
        torch.cuda.synchronize()
        t_fb = (time.perf_counter() - t0) * 1e3 / reps
        pr.assemble(0.0, 0.0)
        pr.gep_slice(a, b, max_slice=P.extra["max_slice"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, U, eta, count, st, stats = pr.gep_slice(a, b, max_slice=P.extra["max_slice"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        good = int(sum(1 for e in eta if e <= 1e-10))
        k = "riga" if s else "iga"
        out[k] = {
            "workload": f"H(curl) p={P.p}, {P.ne}x{P.ne}, perfect conductor, " +
                        (f"rIGA s={s}" if s else "IGA"),
            "ndof": int(pr.ndof), "nnz": int(pr.nnz), "max_front": int(info["max_front"]),
            "factor_gflop_algorithmic": info["factor_flops"] / 1e9, "factor_ms": t_fac,
            "factor_gflops": info["factor_flops"] / (t_fac * 1e-3) / 1e9,
            "solve_2rhs_ms": t_fb, "solve_factor_mb": info["solve_bytes"] / 1e6,
            "maxwell": {"interval": [a, b], "count": int(count), "found": int(len(mu)), "status": int(st),
                        "ms": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
                        "max_eta": float(max(eta)) if len(eta) else None, **stats},
        }
        mus[k] = (P, mu)
        pr.close()
    r, i = out["riga"], out["iga"]
    out["iga_over_riga"] = {
        "factor_flops": i["factor_gflop_algorithmic"] / r["factor_gflop_algorithmic"],
        "factor_time": i["factor_ms"] / r["factor_ms"],
        "fb_bytes": i["solve_factor_mb"] / r["solve_factor_mb"],
        "fb_time": i["solve_2rhs_ms"] / r["solve_2rhs_ms"],
        "mat_vec_nnz": i["nnz"] / r["nnz"], "vec_vec_ndof": i["ndof"] / r["ndof"],
        "maxwell_time": i["maxwell"]["ms"] / r["maxwell"]["ms"],
    }
    return out, mus


def flop_table(riga, nes=(256, 1024), degrees=(3, 4, 5, 6)):
    """Host-only analog of tab:FlopTest for the curl-conforming space with the
    perfect-conductor condition: symbolic factorization flops and nnz(L) of
    the library's elimination order, IGA over rIGA (16 x 16 macroelements),
    and the matrix and vector size ratios."""
    rows = []
    for ne in nes:
        for p in degrees:
            c = {}
            for s in (16, 0):
                order, cc, nz, fl = riga.riga_symbolic(p, ne, s, space=riga.RIGA_SPACE_HCURL)
                c[s] = (len(order), int(nz), fl)
            rows.append({"p": p, "ne": ne, "ndof_riga": c[16][0], "ndof_iga": c[0][0],
                         "factorization": c[0][2] / c[16][2], "fb_elimination": c[0][1] / c[16][1],
                         "vec_vec": c[0][0] / c[16][0]})
            print(json.dumps(rows[-1]), flush=True)
    return rows


def complex_target_form(torch, riga, W, steps, block, cfg=None):
    """A QEP at a complex target, rIGA and IGA: by default the conductive
    electromagnetic QEP on the curl-conforming space (p=3, 256^2, perfect
    conductor) at 7i, else the workload `cfg` gives (the vibroacoustic cavity);
    the real form of Q(sigma) factored by LU, the eigensolve on the real part
    of the operator; one step = assemble + factor + eigensolve, timed like the
    headline step."""
    if cfg is None:
        cfg = W.cfg_em_qep
    out, lams = {}, {}
    for s in (16, 0):
        P = cfg(s)
        pr = riga.Problem(P.p, P.ne, P.hyper_every, space=P.extra["space"], walls=P.extra.get("walls", 0))
        info = pr.info
        sig = P.extra["sigma_c"]

        def one():
            pr.assemble(P.alpha, P.beta)
            pr.factor(sig)
            return pr.eigs(P.nev, P.m, block=block, seed=0, vectors=True)

        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lam, X, eta, nconv, st = one()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        stats = pr.stats()
        good = int(sum(1 for e in eta[:nconv] if e <= 1e-10))
        space = ("H(curl) p={}, {}x{}, perfect conductor".format(P.p, P.ne, P.ne) if P.extra["space"] == 1 else
                 "H(div) p={}, {}x{}, rigid walls, absorbing top wall (alpha {}, beta {})".format(
                     P.p, P.ne, P.ne, P.alpha, P.beta))
        damping = f"C = {P.alpha}M + {P.beta}K, " if P.extra["space"] == 1 else ""
        out["riga" if s else "iga"] = {
            "workload": space + ", " + (f"rIGA s={s}" if s else "IGA") +
                        f", {damping}{P.nev} pairs of largest |psi| at sigma={sig}, subspace {P.m}",
            "ndof": int(info["ndof"]), "ms_per_step": ms, "eigenpairs_per_s": good * 1e3 / ms, "pairs_ok": good,
            "status": int(st), "factor_ms": stats["t_factor_ms"], "eigs_ms": stats["t_eigs_ms"],
            # the real form: twice the unknowns, LU (two triangles) of the doubled fronts
            "factor_gflop_dense": stats["flops"]["factor"] / 1e9,
            "factor_gflops_dense": stats["flops"]["factor"] / (stats["t_factor_ms"] * 1e-3) / 1e9,
            "n_it": int(stats["n_it"]), "n_fb": int(stats["n_fb"]), "max_eta": float(max(eta)),
        }
        lams["riga" if s else "iga"] = (P, lam)
        pr.close()
    r, i = out["riga"], out["iga"]
    out["iga_over_riga"] = {"factor_time": i["factor_ms"] / r["factor_ms"], "eigs_time": i["eigs_ms"] / r["eigs_ms"],
                            "step_time": i["ms_per_step"] / r["ms_per_step"]}
    return out, lams


def flop_test(torch, riga, degrees=(3, 4, 5), ne=256, nev=100, m=220, block=2):
    """tab:FlopTest on the device: the conductive QEP on the curl-conforming
    space with the perfect conductor (C = 0.05 M + 0.005 K, target 7i, nev
    pairs, subspace m), rIGA (16 x 16-element macroelements) against IGA for
    each degree.  Per operation of eq. Cost the ratio IGA / rIGA of the
    library's counts (factorization: the symbolic flops of the elimination
    order; FB elimination: nnz(L) x solves; mat-vec: nnz x products; vec-vec:
    N x products) and of the measured factorization, eigensolve and total
    times (one warm-up, one timed call each)."""
    rows = []
    for p in degrees:
        res = {}
        for s in (16, 0):
            pr = riga.Problem(p, ne, s, space=riga.RIGA_SPACE_HCURL)
            info = pr.info
            _, _, nnz_l, sym_flops = riga.riga_symbolic(p, ne, s, space=riga.RIGA_SPACE_HCURL)
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pr.assemble(0.05, 0.005)
                pr.factor(7.0j)
                lam, X, eta, nconv, st = pr.eigs(nev, m, block=block, seed=0, vectors=False)
                torch.cuda.synchronize()
                total = (time.perf_counter() - t0) * 1e3
            S = pr.stats()
            res[s] = {"ndof": int(info["ndof"]), "nnz": int(info["nnz"]), "nnz_l": int(nnz_l), "sym_flops": sym_flops,
                      "factor_ms": S["t_factor_ms"], "eigs_ms": S["t_eigs_ms"], "total_ms": total,
                      "n_fb": int(S["n_fb"]), "n_mv": int(S["n_mv"]), "n_vv": int(S["n_vv"]), "status": int(st),
                      "nconv": int(nconv), "max_eta": float(max(eta[:max(nconv, 1)]))}
            pr.close()
        r, i = res[16], res[0]
        row = {"p": p, "ne": ne, "nev": nev, "m": m, "riga": r, "iga": i, "iga_over_riga": {
            "factorization_flops": i["sym_flops"] / r["sym_flops"],
            "fb_elimination": (i["nnz_l"] * i["n_fb"]) / (r["nnz_l"] * r["n_fb"]),
            "mat_vec": (i["nnz"] * i["n_mv"]) / (r["nnz"] * r["n_mv"]),
            "vec_vec": (i["ndof"] * i["n_vv"]) / (r["ndof"] * r["n_vv"]),
            "factor_time": i["factor_ms"] / r["factor_ms"], "eigs_time": i["eigs_ms"] / r["eigs_ms"],
            "total_time": i["total_ms"] / r["total_ms"]}}
        rows.append(row)
        print(json.dumps(row), flush=True)
    return rows


def oracle_check_em(lams):
    """Eigenvalues of the complex-target leg against the oracle's Maxwell
    closed form with the null space, selected by |psi|."""
    import numpy as np

    from oracle import cshift

    res = {}
    for k, (P, lam) in lams.items():
        ref = cshift.maxwell_cshift(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.extra["sigma_c"], P.nev)
        rel = np.abs(lam - ref) / np.abs(ref) if len(ref) == len(lam) else np.array([np.inf])
        res[k] = (float(rel.max()), int(np.sum(rel <= 1e-10)))
    return res


def check_vibroacoustic(lams):
    """The vibroacoustic leg has no closed form at full size: every returned
    eigenvalue decays or oscillates without growth (Re lam <= 0, the
    semidefinite K and C of eq. HdivQuadEig) and the set is closed under
    conjugation."""
    import numpy as np

    res = {}
    for k, (P, lam) in lams.items():
        scale = np.abs(lam).max()
        conj_ok = all(np.min(np.abs(lam - np.conj(x))) <= 1e-9 * abs(x) for x in lam[:-2])
        res[k] = {"max_re_over_abs": float(lam.real.max() / scale), "conjugate_closed": bool(conj_ok)}
    return res


def oracle_check_hcurl(mus):
    """Count and eigenvalues of the Maxwell slices of the vector-space leg
    against the oracle's closed form (sums of 1-D values)."""
    import numpy as np

    from oracle import hcurl as ohc

    res = {}
    for k, (P, mu) in mus.items():
        a, b = P.extra["interval"]
        ref = ohc.maxwell_closed(P.p, P.ne, P.hyper_every, True, a, b)
        rel = float(np.max(np.abs(mu - ref) / np.abs(ref))) if len(ref) == len(mu) and len(mu) else None
        res[k] = (len(ref), rel)
    return res


def cpu_baseline(P, lam_gpu):
    """The oracle as it stands: SciPy sparse LU of Q(sigma) + ARPACK on the
    shift-and-invert operator, same workload (full solve, ~30 s)."""
    import numpy as np

    from oracle import assemble as oasm
    from oracle import eigen as oeig

    import scipy

    cores = len(os.sched_getaffinity(0))
    K, M, C = oasm.assemble(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    t0 = time.perf_counter()
    lam = oeig.shift_invert(K, C, M, P.sigma, P.nev)
    t = time.perf_counter() - t0
    rel_gpu, _ = oracle_check(P, lam_gpu)
    blas_threads = os.environ.get("OMP_NUM_THREADS", "unset")
    return {"value": P.nev / t, "unit": "eigenpairs/s", "cores": cores, "kind": "oracle",
            "sample": f"full factor+eigensolve of the same workload (SciPy splu + ARPACK, {P.nev} pairs), "
                      f"{t:.1f} s",
            "blas_threads": blas_threads, "numpy": np.__version__, "scipy": scipy.__version__}, rel_gpu


COPY_BYTES = 512 * 1024 * 1024


def copy_calibration(torch):
    """A plain device-to-device copy of COPY_BYTES, three times: the HBM byte
    counters a profiler reads for it, against the 2 x COPY_BYTES it must move,
    scale the counters of the solver's kernels."""
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": COPY_BYTES, "copies": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--block", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-iga", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-undamped", action="store_true")
    ap.add_argument("--no-toar", action="store_true")
    ap.add_argument("--no-gyro", action="store_true")
    ap.add_argument("--no-hcurl", action="store_true")
    ap.add_argument("--no-em", action="store_true")
    ap.add_argument("--no-vibro", action="store_true")
    ap.add_argument("--flop-test", action="store_true",
                    help="only run the device analog of tab:FlopTest (the conductive QEP on the curl-conforming "
                         "space at the target 7i, 100 pairs, p = 3..5 on 256^2, rIGA against IGA) and exit")
    ap.add_argument("--flop-table", action="store_true",
                    help="only print the host-side symbolic cost ratios IGA / rIGA of the curl-conforming space "
                         "(p = 3..6, 256^2 and 1024^2 elements) and exit")
    ap.add_argument("--basis", choices=("full", "toar"), default="full",
                    help="Krylov basis of the timed headline steps: the full 2N-long basis (default) or the "
                         "compact two-level form")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy three times (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.flop_table:
        from paper_2112_14064_amd import riga
        flop_table(riga)
        return
    if args.flop_test:
        from paper_2112_14064_amd import riga
        riga.load()
        flop_test(torch, riga)
        return

    from paper_2112_14064_amd import riga
    from paper_2112_14064_amd import workloads as W

    riga.load()
    P = W.cfg_riga_vs_iga(16)
    main_flags = riga.RIGA_EIGS_TOAR if args.basis == "toar" else 0
    pr, res, lam = run_config(torch, riga, P, args.steps, args.warmup, args.block, flags=main_flags)
    roof = roofline(pr, res, args.block)
    pr.close()
    iga = None
    if not args.no_iga:
        Pi = W.cfg_riga_vs_iga(0)
        pri, iga, lam_iga = run_config(torch, riga, Pi, 1, 1, args.block, flags=main_flags)
        pri.close()
    out = {
        "metric": METRIC,
        "value": res["eigenpairs_per_s"],
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "damped-wave QEP on the unit square, p=3, 256x256 elements, rIGA C0 "
                               "hyperplanes every 16 elements, Rayleigh 0.05M+0.005K, 40 eigenpairs "
                               "nearest sigma=2, subspace 80",
                   "p": P.p, "ne": P.ne, "hyper_every": P.hyper_every, "nev": P.nev, "m": P.m,
                   "block": args.block, "ndof": res["ndof"], "basis": args.basis},
        "riga_fp64": res,
    }
    if iga is not None:
        out["iga_fp64"] = iga
        out["riga_speedup_vs_iga"] = {
            "factor": iga["factor_ms"] / res["factor_ms"],
            "eigs": iga["eigs_ms"] / res["eigs_ms"],
            "step": iga["ms_per_step"] / res["ms_per_step"],
        }
    gyro_lams = None
    if not args.no_gyro:
        out["gyroscopic_form"], gyro_lams = gyroscopic_form(torch, riga, W, min(args.steps, 3), args.block)
    toar_lams = None
    if not args.no_toar:
        out["compact_basis_form"], toar_lams = compact_basis_form(torch, riga, W, args.steps, args.block)
    if not args.no_mixed:
        out["precision_form"] = precision_form(torch, riga, W)
    if not args.no_batch:
        out["batching_form"] = batching_form(torch, riga, W)
    mus = None
    if not args.no_undamped:
        out["undamped_form"], mus = undamped_form(torch, riga, W)
    hc = None
    if not args.no_hcurl:
        out["vector_space_form"], hc = vector_space_form(torch, riga, W)
    em = None
    if not args.no_em:
        out["complex_target_form"], em = complex_target_form(torch, riga, W, min(args.steps, 2), args.block)
    if not args.no_vibro:
        out["vibroacoustic_form"], vib = complex_target_form(torch, riga, W, min(args.steps, 2), args.block,
                                                             cfg=W.cfg_vibroacoustic)
        for k, v in check_vibroacoustic(vib).items():
            out["vibroacoustic_form"][k].update(v)
    if roof is not None:
        out["roofline"] = roof
    if not args.no_cpu:
        cb, rel = cpu_baseline(P, lam)
        out["cpu_baseline"] = cb
        # the metric's 1e-10 eigenvalue error, checked against the oracle's closed form
        out["riga_fp64"]["max_rel_err_vs_oracle"], out["riga_fp64"]["pairs_within_1e-10_of_oracle"] = \
            oracle_check(P, lam)
        if iga is not None:
            out["iga_fp64"]["max_rel_err_vs_oracle"], out["iga_fp64"]["pairs_within_1e-10_of_oracle"] = \
                oracle_check(Pi, lam_iga)
        if gyro_lams is not None:
            for k, (rel, ok) in oracle_check_gyro(gyro_lams).items():
                out["gyroscopic_form"][k]["max_rel_err_vs_oracle"] = rel
                out["gyroscopic_form"][k]["pairs_within_1e-10_of_oracle"] = ok
        if toar_lams is not None:
            for k, (Pt, lt) in toar_lams.items():
                out["compact_basis_form"][k]["max_rel_err_vs_oracle"], \
                    out["compact_basis_form"][k]["pairs_within_1e-10_of_oracle"] = oracle_check(Pt, lt)
        if mus is not None:
            for k, (n_ref, rel) in oracle_check_undamped(mus).items():
                out["undamped_form"][k]["oracle_count"] = n_ref
                out["undamped_form"][k]["max_rel_err_vs_oracle"] = rel
        if em is not None:
            for k, (rel, ok) in oracle_check_em(em).items():
                out["complex_target_form"][k]["max_rel_err_vs_oracle"] = rel
                out["complex_target_form"][k]["pairs_within_1e-10_of_oracle"] = ok
        if hc is not None:
            for k, (n_ref, rel) in oracle_check_hcurl(hc).items():
                out["vector_space_form"][k]["maxwell"]["oracle_count"] = n_ref
                out["vector_space_form"][k]["maxwell"]["max_rel_err_vs_oracle"] = rel
    print(json.dumps(out))


if __name__ == "__main__":
    main()
