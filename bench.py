#!/usr/bin/env python3
"""Throughput of the density-fitted GW hot path on one MI355X.

One step is one damped scGW iteration of the paper's workflow (Sec. IV.A):
  Sigma[G] + Pi evaluation  (Hartree-Fock, polarization, tau -> i Omega,
                             screened-interaction solve, i Omega -> tau,
                             self-energy; Algorithm 1 over all q)
  + damping of Sigma, Sigma~ tau -> i omega, chemical-potential search
  (Dyson + density at every probe), G i omega -> tau.
The metric is Sigma+Pi evaluations per second (one per step) with the
algorithmic GFLOP/s of the two contraction chains and its fraction of the
fp64 MFMA peak.  Inputs are synthetic (seeded generator) and resident in HBM
before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6       # MI355X dense fp64 matrix peak (AMD specification)
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def contraction_flops(nk, nao, naux, ntau):
    """Algorithmic flops of the polarization and self-energy chains per
    evaluation: 2 Nk^2 Ntau (8 naux^2 nao^2 + 16 naux nao^3)."""
    return 2.0 * nk * nk * ntau * (8.0 * naux ** 2 * nao ** 2 + 16.0 * naux * nao ** 3)


def kernel_source_hash():
    from paper_2206_07660_amd.build import source_hash
    return source_hash()


def load_traffic(kclass_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    c = d.get("classes", {}).get(kclass_name)
    if not c:
        return None
    return c.get("hbm_bytes_per_launch")


def host_info():
    """CPU model, logical CPU count and the BLAS numpy calls (vendor, threads)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        import numpy  # noqa: F401  (loads the BLAS numpy links)
        from threadpoolctl import threadpool_info
        blas = [{k: i.get(k) for k in ("internal_api", "version", "num_threads")}
                for i in threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas}


def oracle_timings():
    """The CPU oracle, as it stands, timed on whole Sigma+Pi evaluations
    (oracle.gw.sigma_evaluation on the G0 of each workload): tiny-2x2x2 with
    all BLAS threads and with one, ad-3x3x3 with all threads."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from paper_2206_07660_amd import inputs as inp
    from oracle import grids as og
    from oracle import gw as ogw
    out = {"host": host_info(), "runs": []}
    for name, threads in (("tiny-2x2x2", None), ("tiny-2x2x2", 1), ("ad-3x3x3", None)):
        wl = inp.WORKLOADS[name]
        g = og.Grids(wl.beta, wl.ntau)
        H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
        G = ogw.g0_tau(H0, S, wl.mu0, wl.beta, g.tau)
        log(f"[oracle] {name}, threads {threads or 'all'}")
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            ogw.sigma_evaluation(V, G, g, wl.mesh, wl.ns)
            dt = time.perf_counter() - t0
        out["runs"].append({"workload": name, "threads": threads or out["host"]["logical_cpus"],
                            "seconds_per_eval": dt,
                            "gflops": contraction_flops(wl.nk, wl.nao, wl.naux, wl.ntau) / dt / 1e9})
        log(f"[oracle] {name}: {dt:.2f} s per evaluation")
    return out


def cpu_baseline(wl, ntau_sample):
    """The CPU oracle, as it stands, timed on this host on a bounded sample of
    the same workload: one q-point, `ntau_sample` tau nodes of the
    polarization and of the self-energy contraction.  Scaled to evaluations/s
    by the share of the full evaluation that the sample is (Nk * ntau / sample)."""
    import numpy as np
    from paper_2206_07660_amd import inputs as inp
    from oracle import gw as ogw
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    Vq = inp.make_V_slab(wl, 0)
    V = np.broadcast_to(Vq[None], (wl.nk,) + Vq.shape)          # only slab q = 0 is read
    rng = np.random.default_rng([wl.seed, 99])
    G = inp.random_hermitian_tau(rng, wl.ntau, wl.nk, wl.nao, 0.1)
    taus = list(range(ntau_sample))
    Pt = inp.circular_gaussian(rng, (1, wl.ntau, wl.naux, wl.naux), 0.01)
    t0 = time.perf_counter()
    ogw.polarization(V, G, wl.mesh, wl.ns, qs=[0], taus=taus)
    t1 = time.perf_counter()
    ogw.self_energy(V, G[:ntau_sample], Pt[:, :ntau_sample], wl.mesh, qs=[0])
    t2 = time.perf_counter()
    t_eval = (t2 - t0) * wl.nk * wl.ntau / ntau_sample
    return {"value": 1.0 / t_eval, "unit": "eval/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"one q-point and {ntau_sample} of {wl.ntau} tau nodes of the polarization "
                       f"and self-energy contractions at the full {wl.name} shape "
                       f"({t1 - t0:.2f} s + {t2 - t1:.2f} s), scaled by Nk*ntau/{ntau_sample}"),
            "seconds_per_eval_extrapolated": t_eval, "host": host_info()}


def mixed_comparison(ctx64, path64, st, V, H0, S, wl, precision="fp32"):
    """One Sigma+Pi evaluation from the current G in fp64 and in a mixed
    path (complex64 V; "fp32": fp32 MFMA contractions, "bf16x3": split-bf16
    MFMA for the two large contractions and fp32 for the producers and the
    final self-energy contraction; fp64 elsewhere): seconds each and the
    max-abs difference of Sigma_inf and Sigma~ in Ha."""
    import torch
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.scgw import GWPath
    G = st.G_tau
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s64_inf, s64_tau = path64.sigma(G)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    ref_inf, ref_tau = s64_inf.clone(), s64_tau.clone()
    V32 = V.to(torch.complex64)
    ctx32 = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, precision=precision)
    p32 = GWPath(ctx32, V32, H0, S, wl.n_target)
    p32.sigma(G)                                   # warm-up
    torch.cuda.synchronize()
    gw.gw_profile_enable(ctx32, True)
    t0 = time.perf_counter()
    s32_inf, s32_tau = p32.sigma(G)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    prof = {n: gw.gw_profile_read(ctx32, kc) for n, kc in gw.KCLASS.items()}
    gw.gw_profile_enable(ctx32, False)
    e_inf = (s32_inf - ref_inf).abs().max().item()
    e_tau = (s32_tau - ref_tau).abs().max().item()
    flops = contraction_flops(wl.nk, wl.nao, wl.naux, wl.ntau)
    n_l, ms_l, fl_l = prof["pol_contract"]
    n_s, ms_s, fl_s = prof["se_contract"]
    how = ("fp32 MFMA with fp64 chunk sums" if precision == "fp32" else
           ("split-bf16 (%s) MFMA for the polarization and P~ V contractions, fp32 MFMA for the "
            "producers and the final self-energy contraction (fp64 chunk sums there; the split "
            "polarization sums its 512-term fp32 chunks in %s)"
            % (precision, "fp32" if precision == "bf16x3" else "fp64")))
    res = {"sigma_eval_s_fp64": t64, "sigma_eval_s_mixed": t32, "speedup": t64 / t32,
           "evals_per_s_mixed": 1.0 / t32,
           "gflops_contractions_mixed": flops / t32 / 1e9,
           "pol_contract_tflops_mixed": fl_l / (ms_l * 1e-3) / 1e12 if ms_l else None,
           "se_contract_tflops_mixed": fl_s / (ms_s * 1e-3) / 1e12 if ms_s else None,
           "max_abs_dSigma_inf_Ha": e_inf, "max_abs_dSigma_tilde_Ha": e_tau,
           "kernel_ms": {k: round(v[1], 2) for k, v in prof.items() if v[0]},
           "precision": "V complex64, G rounded to complex64, " + how +
                        "; transforms, screened-interaction solve, HF, Dyson, mu in fp64"}
    if precision == "fp32":
        res["fp32_mfma_frac_path"] = flops / t32 / 157.3e12
    else:
        # bf16x3 / bf16x6 run three / six bf16 products per real product: the
        # fraction of the dense bf16 MFMA peak (2.5 PFLOP/s) the two split
        # contractions reach, and their rate against the fp32 MFMA peak
        # (157.3 TFLOP/s)
        nprod = 3.0 if precision == "bf16x3" else 6.0
        for name, (n_c, ms_c, fl_c) in (("pol_contract", prof["pol_contract"]), ("se_contract", prof["se_contract"])):
            if ms_c:
                rate = fl_c / (ms_c * 1e-3)
                res[name + "_bf16_mfma_frac"] = nprod * rate / 2.5e15
                res[name + "_vs_fp32_peak"] = rate / 157.3e12
    ctx32.close()
    del V32, p32
    torch.cuda.empty_cache()
    log(f"[bench] mixed {precision}: {t32:.2f} s vs fp64 {t64:.2f} s per Sigma+Pi evaluation, "
        f"max|dSigma| {max(e_inf, e_tau):.2e} Ha")
    return res


def ir_comparison(path, V, H0, S, wl, lam, eps, ms_step_cheb):
    """The same workload on intermediate-representation grids (Sec. IV.C;
    ntau = the IR basis size for lambda, eps): one Sigma+Pi evaluation from G0
    on each grid, one damped scGW step on the IR grids, and how far the two
    representations' Sigma lie apart (Sigma_inf, and Sigma~(i w_n) at the
    Matsubara frequencies both sparse sets hold)."""
    import numpy as np
    import torch
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.scgw import GWPath
    ctx_ir = gw.Context(wl.mesh, wl.nao, wl.naux, None, wl.beta, ns=wl.ns, ir=(lam, eps))
    p_ir = GWPath(ctx_ir, V, H0, S, wl.n_target)
    st_c, st_i = path.start(0.0), p_ir.start(0.0)
    # the same G0 on both grids: Dyson at the chemical potential of the
    # Chebyshev search (in a gap the roots of the two counts differ)
    gw.gw_dyson_G(ctx_ir, H0, S, None, None, st_c.mu, st_i.G_iw)
    gw.gw_iw_to_tau(ctx_ir, gw.GW_FERMION, st_i.G_iw, st_i.G_tau)
    p_ir.sigma(st_i.G_tau)                             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    si_c, ss_c = path.sigma(st_c.G_tau)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    si_c, ss_c = si_c.cpu().numpy(), ss_c.cpu().numpy()
    t0 = time.perf_counter()
    si_i, ss_i = p_ir.sigma(st_i.G_tau)
    torch.cuda.synchronize()
    t_i = time.perf_counter() - t0
    si_i, ss_i = si_i.cpu().numpy(), ss_i.cpu().numpy()
    gc, gi = path.ctx.get_grids(), ctx_ir.get_grids()
    wc = dict(zip(gc["nF"].tolist(), np.tensordot(gc["TF"], ss_c, axes=(1, 0))))
    wi = dict(zip(gi["nF"].tolist(), np.tensordot(gi["TF"], ss_i, axes=(1, 0))))
    common = sorted(set(wc) & set(wi))
    d_iw = max(float(np.abs(wc[n] - wi[n]).max()) for n in common) if common else None
    steps = 2
    p_ir.step(st_i)                                    # warm-up step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p_ir.step(st_i)
    torch.cuda.synchronize()
    ms_ir = 1e3 * (time.perf_counter() - t0) / steps
    # the same IR grids with the split-bf16 contractions (complex64 V)
    G_ir = st_i.G_tau.clone()
    ctx_ir.close()
    del p_ir
    torch.cuda.empty_cache()
    V32 = V.to(torch.complex64)
    ctx_b = gw.Context(wl.mesh, wl.nao, wl.naux, None, wl.beta, ns=wl.ns, ir=(lam, eps), precision="bf16x3")
    p_b = GWPath(ctx_b, V32, H0, S, wl.n_target)
    p_b.sigma(G_ir)                                    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_b.sigma(G_ir)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    ctx_b.close()
    del p_b, V32
    torch.cuda.empty_cache()
    res = {"lambda": lam, "eps": eps, "ntau": ctx_ir.ntau, "nw_f": ctx_ir.nw_f, "nw_b": ctx_ir.nw_b,
           "ntau_chebyshev": path.ctx.ntau,
           "sigma_eval_s_chebyshev": t_c, "sigma_eval_s_ir": t_i, "evals_per_s_ir": 1.0 / t_i,
           "speedup_eval": t_c / t_i, "ms_per_step_ir": ms_ir, "speedup_step": ms_step_cheb / ms_ir,
           "max_abs_dSigma_inf_Ha": float(np.abs(si_c - si_i).max()),
           "max_abs_dSigma_iw_common_Ha": d_iw, "common_frequencies": len(common),
           "sigma_eval_s_ir_bf16x3": t_b, "speedup_eval_ir_bf16x3_over_chebyshev_fp64": t_c / t_b,
           "note": "G0 of H0 at the same mu on each grid; Sigma~(i w) compared where the sparse sets "
                   "share Matsubara indices; the IR step then runs its own mu search; the bf16x3 "
                   "evaluation is on the IR grids from the G of the IR steps"}
    log(f"[bench] IR grids (ntau {res['ntau']}): {t_i:.2f} s vs Chebyshev ({path.ctx.ntau}) {t_c:.2f} s per "
        f"evaluation, step {ms_ir:.0f} ms; max|dSigma| {res['max_abs_dSigma_inf_Ha']:.1e} / {d_iw}; "
        f"IR + bf16x3 {t_b:.2f} s")
    return res


def solve(path, wl, args, start=None):
    """One self-consistent solve to max |Sigma[G(x)] - x| < args.tol from G0
    with the chosen solver on the given path (precision, grids and mu mode
    as built); seconds, evaluations, residual history, mu and N_e."""
    import torch
    from paper_2206_07660_amd.diis import DIIS
    from paper_2206_07660_amd.newton import NewtonKrylov
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = begin(path, start)
    deadline = t0 + args.max_seconds if args.max_seconds else None
    out = {"solver": args.solve, "mu0": st.mu}
    if args.solve == "damped":
        res = []
        for _ in range(args.max_evals):
            path.step(st)
            res.append(st.dsig)
            log(f"[solve] damped {len(res)}: dSigma {st.dsig:.3e} mu {st.mu:.10f} N_e {st.n_e:.12f}")
            if st.dsig < args.tol or (deadline and time.perf_counter() > deadline):
                break
        out.update(evaluations=len(res), residuals=res, mu=st.mu, n_e=st.n_e)
    elif args.solve == "diis":
        dz = DIIS(path, depth=6)
        x, F = dz.solve(st.sig_inf, st.sig_tau, st.mu, tol=args.tol, max_iter=args.max_evals,
                        log=lambda m: log(f"[solve] {m}"), deadline=deadline)
        out.update(evaluations=dz.stats.evaluations, residuals=dz.stats.residuals, mu=dz.mu,
                   n_e=dz.n_e)
    else:
        if start is None:
            for _ in range(2):
                path.step(st)
        nk = NewtonKrylov(path, restart=20, gmres_rtol=1e-3, per_q=args.per_q,
                          log=lambda m: log(f"[solve] {m}"))
        x, F = nk.solve(st.sig_inf, st.sig_tau, st.mu, tol=args.tol, max_steps=args.max_evals,
                        log=lambda m: log(f"[solve] {m}"), deadline=deadline)
        out.update(evaluations=nk.stats.evaluations + (2 if start is None else 0), jvps=nk.stats.jvps,
                   newton_steps=nk.stats.newton_steps, residuals=nk.stats.residuals, mu=nk.mu)
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    out["final_residual_Ha"] = out["residuals"][-1] if out["residuals"] else None
    out["converged"] = bool(out["final_residual_Ha"] is not None and out["final_residual_Ha"] < args.tol)
    return out


def compare_solvers(path, wl, tol):
    """Damped fixed point, Pulay DIIS and Newton-Krylov (GMRES(20)) to
    max |Sigma[G(x)] - x| < tol, all on the fp64 path; the fixed point and
    DIIS start from G0, Newton-Krylov after two damped steps from G0."""
    import torch
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.diis import DIIS
    from paper_2206_07660_amd.newton import NewtonKrylov
    flops = contraction_flops(wl.nk, wl.nao, wl.naux, wl.ntau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = path.start(0.0)
    n_fp = 0
    while n_fp < 300:
        path.step(st)
        n_fp += 1
        log(f"[solvers] fixed point {n_fp}: dSigma {st.dsig:.3e}")
        if st.dsig < tol:
            break
    torch.cuda.synchronize()
    t_fp = time.perf_counter() - t0
    fp_inf, fp_tau = st.sig_inf.clone(), st.sig_tau.clone()
    t0 = time.perf_counter()
    st2 = path.start(0.0)
    for _ in range(2):
        path.step(st2)
    nk = NewtonKrylov(path, restart=20, gmres_rtol=1e-3)
    x, F = nk.solve(st2.sig_inf, st2.sig_tau, st2.mu, tol=tol, max_steps=30, log=log)
    torch.cuda.synchronize()
    t_nk = time.perf_counter() - t0
    d = max((nk.inf(x) - fp_inf).abs().max().item(), (nk.tau(x) - fp_tau).abs().max().item())
    # the same Newton-Krylov solve with P~ rebuilt per q inside each derivative
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st3 = path.start(0.0)
    for _ in range(2):
        path.step(st3)
    nkq = NewtonKrylov(path, restart=20, gmres_rtol=1e-3, per_q=True)
    xq, Fq = nkq.solve(st3.sig_inf, st3.sig_tau, st3.mu, tol=tol, max_steps=30, log=log)
    torch.cuda.synchronize()
    t_nkq = time.perf_counter() - t0
    dq = max((nkq.inf(xq) - nk.inf(x)).abs().max().item(), (nkq.tau(xq) - nk.tau(x)).abs().max().item())
    # Pulay DIIS on the same residual, from the same start as the fixed point
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st4 = path.start(0.0)
    dz = DIIS(path, depth=6)
    xd, Fd = dz.solve(st4.sig_inf, st4.sig_tau, st4.mu, tol=tol, max_iter=100, log=log)
    torch.cuda.synchronize()
    t_diis = time.perf_counter() - t0
    dd = max((dz.inf(xd) - fp_inf).abs().max().item(), (dz.tau(xd) - fp_tau).abs().max().item())
    return {"metric": "scGW solve to equal residual: damped fixed point vs DIIS vs Newton-Krylov (fp64)",
            "workload": wl.name, "tol_max_abs_residual_Ha": tol,
            "fixed_point": {"iterations": n_fp, "sigma_evaluations": n_fp, "seconds": t_fp,
                            "final_dsigma": st.dsig},
            "newton_krylov": {"newton_steps": nk.stats.newton_steps,
                              "sigma_evaluations": nk.stats.evaluations + 2,
                              "jvps": nk.stats.jvps, "seconds": t_nk,
                              "residuals": nk.stats.residuals},
            "newton_krylov_per_q_recompute": {"newton_steps": nkq.stats.newton_steps,
                                              "sigma_evaluations": nkq.stats.evaluations + 2,
                                              "jvps": nkq.stats.jvps, "seconds": t_nkq,
                                              "max_abs_sigma_difference_vs_stored_Ha": dq},
            "diis": {"depth": dz.core.depth, "iterations": dz.stats.iterations,
                     "sigma_evaluations": dz.stats.evaluations, "seconds": t_diis,
                     "residuals": dz.stats.residuals, "max_abs_sigma_difference_vs_fixed_point_Ha": dd},
            "speedup_nk_over_fixed_point": t_fp / t_nk,
            "speedup_diis_over_fixed_point": t_fp / t_diis,
            "speedup_nk_over_diis": t_diis / t_nk,
            "max_abs_sigma_difference_Ha": d,
            "gflop_per_sigma_evaluation": flops / 1e9}


def presolve(path, tol, max_evals=40):
    """Canonical DIIS (mu searched for N_target at every residual) from G0 to
    max |F| < tol; returns copies of (Sigma_inf, Sigma~(tau)) and mu.  It
    fixes the chemical potential of the grand-canonical solves that follow."""
    from paper_2206_07660_amd.diis import DIIS
    keep = path.fixed_mu
    path.fixed_mu = False
    try:
        s0 = path.start(0.0)
        dz = DIIS(path, depth=6)
        x, F = dz.solve(s0.sig_inf, s0.sig_tau, s0.mu, tol=tol, max_iter=max_evals,
                        log=lambda m: log(f"[presolve] {m}"))
    finally:
        path.fixed_mu = keep
    return dz.inf(x).clone(), dz.tau(x).clone(), dz.mu, dz.stats.evaluations


def begin(path, start):
    """Scheme start: G0 at the mu of N_target (start None), or the state
    (Sigma_inf, Sigma~, mu) of a pre-solve with its G at that mu."""
    from paper_2206_07660_amd import gw
    if start is None:
        return path.start(0.0)
    st = path.start(start[2], search=False)
    gw.gw_axpby(path.ctx, 1.0, start[0], 0.0, st.sig_inf)
    gw.gw_axpby(path.ctx, 1.0, start[1], 0.0, st.sig_tau)
    gw.gw_tau_to_iw(path.ctx, gw.GW_FERMION, st.sig_tau, path.sig_iw)
    st.mu, st.n_e = path.green(st.sig_inf, path.sig_iw, start[2], st.G_iw, st.G_tau)
    return st


def compare_precisions(path64, V, H0, S, wl, tol, presolve_tol=1e-4):
    """Whole self-consistent solves to max |Sigma[G(x)] - x| < tol: the plain
    damped fp64 loop, DIIS and Newton-Krylov in fp64 and DIIS in the mixed
    path (complex64 V; fp32 MFMA and split-bf16 bf16x3 contractions); seconds, evaluations, and how
    far the fixed points lie apart (equal-accuracy check).  With a
    grand-canonical path64 (fixed_mu) every solver starts from one canonical
    DIIS pre-solve to presolve_tol and holds its mu, so that all of them
    converge to the same self-energy; otherwise each starts from G0 and
    searches mu at every residual."""
    import torch
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.diis import DIIS
    from paper_2206_07660_amd.newton import NewtonKrylov
    from paper_2206_07660_amd.scgw import GWPath
    fixed = bool(path64.fixed_mu)
    out = {"metric": "scGW solve to equal residual: plain fp64 loop vs DIIS and Newton-Krylov fp64 vs "
                     "DIIS mixed",
           "workload": wl.name, "tol_max_abs_residual_Ha": tol, "fixed_mu": fixed}
    ctx32 = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, precision="fp32")
    p32 = GWPath(ctx32, V.to(torch.complex64), H0, S, wl.n_target, fixed_mu=fixed)
    ctxbf = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, precision="bf16x3")
    pbf = GWPath(ctxbf, p32.V, H0, S, wl.n_target, fixed_mu=fixed)
    start = None
    if fixed:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        si, stau, mu, nev = presolve(path64, presolve_tol)
        start = (si, stau, mu)
        out["presolve"] = {"solver": "canonical DIIS (fp64)", "tol": presolve_tol, "sigma_evaluations": nev,
                           "seconds": time.perf_counter() - t0, "mu": mu}
    sols = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = begin(path64, start)
    n_fp = 0
    while n_fp < 80:
        path64.step(st)
        n_fp += 1
        log(f"[precisions] fp64 damped {n_fp}: dSigma {st.dsig:.3e} mu {st.mu:.10f} N_e {st.n_e:.10f}")
        if st.dsig < tol:
            break
    torch.cuda.synchronize()
    out["fp64_damped"] = {"iterations": n_fp, "sigma_evaluations": n_fp,
                          "seconds": time.perf_counter() - t0, "final_dsigma": st.dsig, "mu": st.mu,
                          "n_e": st.n_e}
    sols["fp64_damped"] = (st.sig_inf.clone(), st.sig_tau.clone())
    for name, p in (("fp64_diis", path64), ("mixed_diis", p32), ("bf16x3_diis", pbf)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s0 = begin(p, start)
        dz = DIIS(p, depth=6)
        x, F = dz.solve(s0.sig_inf, s0.sig_tau, s0.mu, tol=tol, max_iter=60,
                        log=lambda m, n=name: log(f"[precisions] {n} {m}"))
        torch.cuda.synchronize()
        sols[name] = (dz.inf(x).clone(), dz.tau(x).clone())
        out[name] = {"iterations": dz.stats.iterations, "sigma_evaluations": dz.stats.evaluations,
                     "seconds": time.perf_counter() - t0, "residuals": dz.stats.residuals, "mu": dz.mu,
                     "n_e": dz.n_e}
    # Newton-Krylov (GMRES(20), stored P~) on the fp64 path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s0 = begin(path64, start)
    nev0 = 0
    if start is None:
        for _ in range(2):
            path64.step(s0)
        nev0 = 2
    nk = NewtonKrylov(path64, restart=20, gmres_rtol=1e-3)
    x, F = nk.solve(s0.sig_inf, s0.sig_tau, s0.mu, tol=tol, max_steps=12,
                    log=lambda m: log(f"[precisions] nk {m}"))
    torch.cuda.synchronize()
    sols["fp64_nk"] = (nk.inf(x).clone(), nk.tau(x).clone())
    out["fp64_nk"] = {"newton_steps": nk.stats.newton_steps, "sigma_evaluations": nk.stats.evaluations + nev0,
                      "jvps": nk.stats.jvps, "seconds": time.perf_counter() - t0,
                      "residuals": nk.stats.residuals, "mu": nk.mu}
    d = lambda a, b: max((a[0] - b[0]).abs().max().item(), (a[1] - b[1]).abs().max().item())
    ref = sols["fp64_damped"]
    out["max_abs_sigma_fp64_diis_vs_damped_Ha"] = d(sols["fp64_diis"], ref)
    out["max_abs_sigma_fp64_nk_vs_damped_Ha"] = d(sols["fp64_nk"], ref)
    out["max_abs_sigma_mixed_vs_fp64_Ha"] = d(sols["mixed_diis"], sols["fp64_diis"])
    out["max_abs_sigma_bf16x3_vs_fp64_Ha"] = d(sols["bf16x3_diis"], sols["fp64_diis"])
    for k in ("fp64_diis", "mixed_diis", "bf16x3_diis", "fp64_nk"):
        out[f"speedup_{k}_over_damped"] = out["fp64_damped"]["seconds"] / out[k]["seconds"]
    out["speedup_mixed_over_fp64_diis"] = out["fp64_diis"]["seconds"] / out["mixed_diis"]["seconds"]
    out["speedup_bf16x3_over_fp64_diis"] = out["fp64_diis"]["seconds"] / out["bf16x3_diis"]["seconds"]
    ctxbf.close()
    ctx32.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="si-4x4x4")
    ap.add_argument("--cpu-sample-tau", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision (fp32 MFMA) comparison")
    ap.add_argument("--no-ir", action="store_true",
                    help="skip the comparison with intermediate-representation grids")
    ap.add_argument("--ir-wmax", type=float, default=5.0,
                    help="omega_max (Ha) of the IR grids: lambda = beta omega_max")
    ap.add_argument("--ir-eps", type=float, default=1e-12)
    ap.add_argument("--compare-solvers", action="store_true",
                    help="instead of the step benchmark: damped fixed point vs DIIS vs Newton-Krylov "
                         "to the same residual (default workload ad-3x3x3)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--compare-precisions", action="store_true",
                    help="instead of the step benchmark: plain fp64 damped loop vs DIIS in fp64 "
                         "and in mixed precision to --tol-mixed (default workload si-4x4x4)")
    ap.add_argument("--tol-mixed", type=float, default=1e-6)
    ap.add_argument("--fixed-mu", action="store_true",
                    help="grand-canonical solves: mu found for N_target at G0, then held")
    ap.add_argument("--solve", choices=["damped", "diis", "nk"],
                    help="instead of the step benchmark: one self-consistent solve to --tol")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3", "bf16x6"], default="fp64",
                    help="precision of the --solve path")
    ap.add_argument("--ir", action="store_true", help="--solve on IR grids (lambda = beta * --ir-wmax)")
    ap.add_argument("--per-q", action="store_true", help="Newton-Krylov with P~ rebuilt per q")
    ap.add_argument("--max-evals", type=int, default=40)
    ap.add_argument("--presolve-tol", type=float, default=1e-4,
                    help="with --fixed-mu: canonical DIIS to this residual fixes mu")
    ap.add_argument("--presolve-max-evals", type=int, default=40)
    ap.add_argument("--max-seconds", type=float, default=0.0)
    ap.add_argument("--oracle-timings", action="store_true",
                    help="instead of the step benchmark: time whole oracle evaluations on the CPU "
                         "(tiny-2x2x2 all threads and one thread, ad-3x3x3 all threads)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the path shards over q across GPUs by design but no multi-GPU run is built.",
              file=sys.stderr)
        sys.exit(2)

    if args.oracle_timings:
        print(json.dumps(oracle_timings()), flush=True)
        return

    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd import inputs as inp
    from paper_2206_07660_amd.scgw import GWPath

    if args.compare_solvers and args.workload == "si-4x4x4":
        args.workload = "ad-3x3x3"
    wl = inp.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] workload {wl.name}: mesh {wl.mesh} nao {wl.nao} naux {wl.naux} ntau {wl.ntau} "
        f"beta {wl.beta}")
    t0 = time.time()
    H0 = torch.from_numpy(inp.make_H0(wl)).to(dev)
    S = torch.from_numpy(inp.make_S(wl)).to(dev)
    vdt = torch.complex64 if (args.solve and args.precision != "fp64") else torch.complex128
    V = torch.empty((wl.nk, wl.nk, wl.naux, wl.nao, wl.nao), dtype=vdt, device=dev)
    nthr = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(nthr) as ex:
        for q, slab in enumerate(ex.map(lambda q: inp.make_V_slab(wl, q), range(wl.nk))):
            V[q].copy_(torch.from_numpy(slab))
    torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM ({V.numel() * V.element_size() / 1e9:.2f} GB V) after "
        f"{time.time() - t0:.1f} s")
    if args.solve:
        ctx = gw.Context(wl.mesh, wl.nao, wl.naux, None if args.ir else wl.ntau, wl.beta, ns=wl.ns,
                         precision=args.precision, ir=(wl.beta * args.ir_wmax, args.ir_eps) if args.ir else None)
        path = GWPath(ctx, V, H0, S, wl.n_target, alpha=0.5, fixed_mu=args.fixed_mu)
        start, pre = None, None
        if args.fixed_mu:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            si, stau, mu, nev = presolve(path, args.presolve_tol, args.presolve_max_evals)
            start = (si, stau, mu)
            pre = {"solver": "canonical DIIS", "tol": args.presolve_tol, "sigma_evaluations": nev,
                   "seconds": time.perf_counter() - t0, "mu": mu}
        res = solve(path, wl, args, start)
        res["presolve"] = pre
        res.update(workload=wl.name, precision=args.precision, fixed_mu=args.fixed_mu,
                   grids=("IR lambda %g eps %g" % (wl.beta * args.ir_wmax, args.ir_eps)) if args.ir
                   else "Chebyshev", ntau=ctx.ntau, tol=args.tol, n_target=wl.n_target)
        print(json.dumps(res), flush=True)
        ctx.close()
        return

    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns)
    log(f"[bench] grids built, tau chunk {ctx.tau_chunk}, workspace "
        f"{ctx.workspace.numel() / 1e9:.1f} GB after {time.time() - t0:.1f} s")
    path = GWPath(ctx, V, H0, S, wl.n_target, alpha=0.5,
                  fixed_mu=args.fixed_mu and (args.compare_solvers or args.compare_precisions))
    if args.compare_solvers:
        print(json.dumps(compare_solvers(path, wl, args.tol)), flush=True)
        ctx.close()
        return
    if args.compare_precisions:
        print(json.dumps(compare_precisions(path, V, H0, S, wl, args.tol_mixed, args.presolve_tol)), flush=True)
        ctx.close()
        return
    st = path.start(0.0)
    log(f"[bench] G0: mu {st.mu:.6f} N_e {st.n_e:.12f}")
    for i in range(args.warmup):
        path.step(st)
        log(f"[bench] warmup {i + 1}/{args.warmup}: mu {st.mu:.8f} N_e {st.n_e:.10f} dSigma {st.dsig:.3e}")
    torch.cuda.synchronize()
    gw.gw_profile_enable(ctx, True)
    hist = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        path.step(st)
        hist.append(dict(mu=st.mu, n_e=st.n_e, dsigma=st.dsig))
        log(f"[bench] step {i + 1}/{args.steps}: mu {st.mu:.8f} N_e {st.n_e:.10f} dSigma {st.dsig:.3e} "
            f"({time.perf_counter() - t_start:.1f} s)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = {name: gw.gw_profile_read(ctx, kc) for name, kc in gw.KCLASS.items()}
    gw.gw_profile_enable(ctx, False)

    ms_step = 1e3 * elapsed / args.steps
    flops = contraction_flops(wl.nk, wl.nao, wl.naux, wl.ntau)
    gflops_nominal = flops / (ms_step * 1e-3) / 1e9
    # flops the contraction kernels executed (P0 is Hermitian for the Hermitian
    # G of the loop, so only its upper tiles are contracted)
    chain = ("pol_contract", "pol_producer", "se_contract", "se_producer", "se_final")
    executed = sum(prof[n][2] for n in chain) / args.steps
    gflops = executed / (ms_step * 1e-3) / 1e9
    dom = max(("pol_contract", "se_contract"), key=lambda n: prof[n][1])
    n_l, ms_l, fl_l = prof[dom]
    achieved = fl_l / (ms_l * 1e-3) / 1e12 if ms_l > 0 else 0.0
    # the same launches on the conventional count, 8 real flops per complex
    # multiply-add (the profiler counts the MFMA flops executed: 6 per complex
    # multiply-add on the three-product form of the fp64 contractions)
    outs = wl.naux * wl.naux if dom == "se_contract" else 0.5 * wl.naux * (wl.naux + 1)
    nominal_l = 8.0 * outs * wl.nk * wl.nao ** 2 * wl.nk * wl.ntau * args.steps / max(n_l, 1)
    exec_ratio = (fl_l / max(n_l, 1)) / nominal_l
    traffic = load_traffic(dom)
    kernel_ms = {k: round(v[1] / args.steps, 3) for k, v in prof.items() if v[0]}
    out = {
        "metric": "Sigma+Pi evaluations/s (fp64), with GFLOP/s and fraction of fp64 MFMA peak",
        "value": 1e3 / ms_step,
        "unit": "eval/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": None,                      # one GPU: no scaling regime
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "mesh": list(wl.mesh), "nk": wl.nk, "nao": wl.nao,
                   "naux": wl.naux, "ntau": wl.ntau, "nw_f": wl.nw_f, "nw_b": wl.nw_b,
                   "beta": wl.beta, "ns": wl.ns, "n_target": wl.n_target, "damping": 0.5,
                   "V": f"complex128 {V.numel() * 16 / 1e9:.2f} GB", "tau_chunk": ctx.tau_chunk,
                   "step": "one damped scGW iteration = one Sigma+Pi evaluation + mu search + Dyson"},
        "gflops_contractions": gflops,
        "mfma_frac_path": gflops / (FP64_MFMA_PEAK_TFLOPS * 1e3),
        "gflops_contractions_nominal": gflops_nominal,
        "nominal_flops_note": "2 Nk^2 ntau (8 naux^2 nao^2 + 16 naux nao^3) per evaluation over the "
                              "step time; counts the full P0 although only its upper tiles are contracted",
        "kernel_ms_per_step": kernel_ms,
        "roofline": {"kernel": f"zgemm_k ({dom})", "bound": "mfma", "achieved": achieved,
                     "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
                     "traffic": traffic, "launches": n_l,
                     "avg_launch_ms": ms_l / max(n_l, 1),
                     "flops_per_launch": fl_l / max(n_l, 1),
                     "flops_basis": ("MFMA flops executed: three-product (Gauss) complex form, 6 real flops "
                                     "per complex multiply-add" if abs(exec_ratio - 0.75) < 1e-9 else
                                     "8 real flops per complex multiply-add"),
                     "flops_per_launch_8flop": nominal_l,
                     "achieved_8flop_equiv": achieved / exec_ratio},
        "history": hist,
    }
    if not args.no_mixed:
        out["mixed_fp32"] = mixed_comparison(ctx, path, st, V, H0, S, wl, "fp32")
        out["mixed_bf16x3"] = mixed_comparison(ctx, path, st, V, H0, S, wl, "bf16x3")
        out["mixed_bf16x6"] = mixed_comparison(ctx, path, st, V, H0, S, wl, "bf16x6")
    if not args.no_ir:
        out["ir_grids"] = ir_comparison(path, V, H0, S, wl, wl.beta * args.ir_wmax, args.ir_eps, ms_step)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_tau)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
