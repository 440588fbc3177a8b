#!/usr/bin/env python
"""Benchmark of the LT-AC G0W0 hot path on one MI355X.

One step = one whole G0W0 evaluation through the C ABI (gw_g0w0): NAF
compression of the raw RI tensors, grids, Laplace-transformed
polarizability, screening, diagonal self-energy, Pade continuation and the
QP solve, with the seeded synthetic inputs already resident in HBM.  The
default workload is the ~2500-basis-function configuration (n_occ = 300
with 80 frozen, n_virt = 2200, n_aux = 7000 -> ~3500 NAFs, 12 Laplace
points, 80 frequencies, 20 QP states) in FP32, generated on the device.

Prints one JSON line: G0W0 wall time per step (value), the live
HIP-event roofline of the dominant kernel (the polarizability SYRK), the
self-energy contraction's rate, the FP64 and BF16x3 paths' wall times for
comparison, the QP errors against the stored FP64 oracle values, the
oracle's CPU time on a bounded sample and, under "paper_scale", one
streamed step of the ~7400-basis-function workload (FP32) when the time
budget allows it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HARTREE_MEV = 27211.386245988
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0}
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_rate(gw, ctx, name):
    ms, n, flops, nbytes = gw.gw_profile_get(ctx, name)
    if n == 0:
        return None
    avg_s = ms / n / 1e3
    return {"launches": n, "avg_ms": ms / n, "flops_per_launch": flops / n,
            "bytes_per_launch": nbytes / n, "tflops": flops / n / avg_s / 1e12,
            "gbs": nbytes / n / avg_s / 1e9}


def source_hash(path):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the stored PMC passes (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy), or None if none were taken for this
    kernel and workload or the kernel's source text (the function the record
    names, hashed) changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}@{workload}")
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src):
        return None
    text = open(src).read()
    i = text.find(rec["region_start"])
    if i < 0:
        return None
    region = text[i:text.index("\n}\n", i) + 3]
    import hashlib
    if hashlib.sha256(region.encode()).hexdigest() != rec["region_sha256"]:
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(prob, torch, n_freq_sample=2, row_frac=0.2, qp_sample=1):
    """Oracle (FP64 NumPy) on a bounded sample of the step (10-30 s on the
    box's host cores), extrapolated to the whole step; no Laplace transform.
    Sample: the NAF metric of the rows of the first ~20% of the occupied
    orbitals (the metric is a sum over rows), the full A x A
    eigendecomposition, the transformation of those rows and of one QP
    state's rows, and per frequency the sum-over-states Pi of those rows, the
    dense inverse of 1 - Pi and W_nm of one QP state, at `n_freq_sample`
    frequencies; each part is scaled by the fraction of rows, states and
    frequencies it covered."""
    from threadpoolctl import threadpool_info
    from oracle import grids, naf, rpa
    c = prob.cfg
    o, v, A = c.n_act_occ, c.n_virt, c.n_aux
    ci = max(1, int(round(o * row_frac)))
    host = lambda t: t.double().cpu().numpy() if hasattr(t, "cpu") else np.asarray(t, np.float64)  # noqa: E731
    R_oo = host(prob.R_oo[:ci])
    R_ov = host(prob.R_ov[:ci * v])
    R_qp = host(prob.R_qp[:qp_sample])
    timing = {}
    t0 = time.perf_counter()
    K = naf.naf_metric(R_oo, R_ov)
    timing["metric"] = (time.perf_counter() - t0) * o / ci
    t0 = time.perf_counter()
    _, U = naf.naf_basis(K, c.eps_naf, c.max_keep)
    timing["eigh"] = time.perf_counter() - t0
    del K
    t0 = time.perf_counter()
    Rt_ov = naf.naf_transform(R_ov, U)
    t_ov = time.perf_counter() - t0
    t0 = time.perf_counter()
    Rt_qp = naf.naf_transform(R_qp, U)
    timing["transform"] = t_ov * o / ci + (time.perf_counter() - t0) * c.n_qp / qp_sample
    om, _ = grids.modified_gauss_legendre(c.n_freq, c.x0)
    sel = om[np.unique(np.linspace(0, len(om) - 1, n_freq_sample).astype(int))]
    d = rpa.delta_ov(prob.eps, c.n_fc, c.n_occ)[:ci * v]
    t0 = time.perf_counter()
    Pi = rpa.pi_sos(Rt_ov, d, sel)
    t_pi = time.perf_counter() - t0
    t0 = time.perf_counter()
    What = rpa.screen(Pi)
    t_inv = time.perf_counter() - t0
    t0 = time.perf_counter()
    W = rpa.w_diag(Rt_qp, What)
    t_w = time.perf_counter() - t0
    assert np.all(np.isfinite(W))
    scale_f = c.n_freq / len(sel)
    timing["pi_sos"] = t_pi * o / ci * scale_f
    timing["inverse"] = t_inv * scale_f
    timing["w_nm"] = t_w * c.n_qp / qp_sample * scale_f
    measured = (timing["metric"] * ci / o + timing["eigh"] + t_ov +
                (timing["transform"] - t_ov * o / ci) * qp_sample / c.n_qp + t_pi + t_inv + t_w)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": round(sum(timing.values()), 3), "unit": "s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"rows of occupied orbitals 0..{ci - 1} of {o} ({ci * (o + v)} of "
                       f"{o * (o + v)} metric rows), the full {A} x {A} eigendecomposition, "
                       f"{qp_sample} of {c.n_qp} QP states, {len(sel)} of {c.n_freq} "
                       f"frequencies; each part scaled by the fraction it covered; sum over "
                       f"states (no Laplace transform)"),
            "measured_s": round(measured, 3),
            "parts_s": {k: round(val, 3) for k, val in timing.items()},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def run_streamed(args, cfg, gw, torch):
    """The paper-scale workload, whose raw tensors do not fit in HBM: the
    occupied-occupied and occupied-virtual rows are generated on the device
    in occupied-index chunks and streamed through the chunked calls twice
    (metric accumulation, then NAF transform and Laplace polarizability
    accumulation), with the requested precisions in lockstep on each chunk
    (the BF16x3 path shares the FP32 path's NAF basis, as in gw_g0w0).
    Screening and self-energy run in frequency batches.  Stage times are
    device-synchronised host times; generation is timed apart and excluded."""
    from gwsynth.device import make_problem_device
    precs = args.precs.split(",")
    c = cfg
    o, v, A, Q, Mo, L, F, Pd = (c.n_act_occ, c.n_virt, c.n_aux, c.n_qp, c.n_act, c.n_lt,
                                c.n_freq, c.n_pade)
    f64 = torch.float64
    t0 = time.perf_counter()
    p = make_problem_device(cfg, "cuda", f64, with_ov=False, with_oo=False, haar_on_device=True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    log(f"{cfg.name}: energies, U and QP rows generated in {gen_s:.1f} s")
    ctx = gw.Context(0)
    # one pass over each shape: autotuning trials would be paid inside the
    # timed stages, so the occupancy-based launch shapes are used
    gw.gw_autotune(ctx, 0)
    chunk = args.chunk_i or max(1, int(args.chunk_gb * 1e9 // ((v + o) * A * 8)))
    mprec = {q: ("fp64" if q == "fp64" else "fp32") for q in precs}
    metric_precs = sorted(set(mprec.values()))
    times = {q: {} for q in set(precs) | set(metric_precs)}

    def timed(q, stage, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        times[q][stage] = times[q].get(stage, 0.0) + time.perf_counter() - t
        return r

    def gen(fn):
        nonlocal gen_s
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        gen_s += time.perf_counter() - t
        return r

    K = {m: torch.zeros((A, A), dtype=f64, device="cuda") for m in metric_precs}
    U = {m: torch.zeros((A, A), dtype=f64, device="cuda") for m in metric_precs}
    for i0 in range(0, o, chunk):
        i1 = min(o, i0 + chunk)
        oo = gen(lambda: p.oo_chunk(i0, i1, f64))
        ov = gen(lambda: p.ov_chunk(i0, i1, f64))
        for m in metric_precs:
            a, b = (oo, ov) if m == "fp64" else (gen(lambda: oo.float()), gen(lambda: ov.float()))
            timed(m, "naf_metric", lambda: gw.gw_naf_compress(ctx, m, A, a, b, K[m], i0 > 0, 0,
                                                              0.0, 0, None))
            del a, b
        del oo, ov
        log(f"metric pass: occupied {i1}/{o}")
    n_naf = {}
    for m in metric_precs:
        n_naf[m], _ = timed(m, "naf_eig", lambda: gw.gw_naf_compress(
            ctx, m, A, None, None, K[m], 1, 1, c.eps_naf, c.max_keep, U[m],
            want_eigvals=False))
        log(f"{m} NAF: {n_naf[m]} of {A} kept")
    del K
    om, wom = gw.gw_freq_grid_mgl(F, c.x0)
    omp, _ = gw.gw_freq_grid_mgl(Pd, c.x0)
    eF, ymin, ymax = gw.gw_prepare(c.n_occ, c.n_fc, c.n_virt, p.eps, om[0])
    x, w, lt_err = gw.gw_lt_grid_minimax(L, ymin, ymax)
    eps_i, eps_a, eps_m = p.eps[c.n_fc:c.n_occ], p.eps[c.n_occ:], p.eps[c.n_fc:]
    ld = {m: (n_naf[m] + 127) // 128 * 128 for m in metric_precs}
    M = {q: torch.zeros((L, n_naf[mprec[q]], n_naf[mprec[q]]), dtype=f64, device="cuda")
         for q in precs}
    for i0 in range(0, o, chunk):
        i1 = min(o, i0 + chunk)
        ov = gen(lambda: p.ov_chunk(i0, i1, f64))
        for m in metric_precs:
            Rin = ov if m == "fp64" else gen(lambda: ov.float())
            Rt = torch.empty((Rin.shape[0], ld[m]), dtype=Rin.dtype, device="cuda")
            timed(m, "naf_transform", lambda: gw.gw_naf_apply(ctx, m, A, n_naf[m], U[m], Rin, Rt))
            del Rin
            for q in precs:
                if mprec[q] != m:
                    continue
                N = n_naf[m]
                timed(q, "chi", lambda: gw.gw_polarizability_lt(
                    ctx, q, N, x, w, i1 - i0, v, eps_i[i0:i1], eps_a, Rt[:, :N], i0 > 0,
                    i1 == o, M[q]))
            del Rt
        del ov
        log(f"polarizability pass: occupied {i1}/{o}")
    Rt_qps = {}
    for m in metric_precs:
        Rqp = p.R_qp if m == "fp64" else p.R_qp.float()
        Rt_qps[m] = torch.empty((Q, Mo, ld[m]), dtype=Rqp.dtype, device="cuda")
        timed(m, "naf_transform", lambda: gw.gw_naf_apply(ctx, m, A, n_naf[m], U[m], Rqp,
                                                          Rt_qps[m]))
        del Rqp
    del U
    torch.cuda.empty_cache()
    out = {}
    for q in precs:
        m = mprec[q]
        N = n_naf[m]
        Rt_qp = Rt_qps[m]
        esz = 8 if q == "fp64" else 4
        fb = max(1, min(F, int(args.screen_gb * 1e9 // (N * N * (esz + (0 if q == "fp64" else 8))))))
        sig = torch.zeros((Q, Pd, 2), dtype=f64, device="cuda")
        for j0 in range(0, F, fb):
            j1 = min(F, j0 + fb)
            W = torch.empty((j1 - j0, N, N), dtype=f64 if q == "fp64" else torch.float32,
                            device="cuda")
            timed(q, "screen", lambda: gw.gw_screen(ctx, q, N, x, M[q], om[j0:j1], W))
            timed(q, "sigma", lambda: gw.gw_sigma_diag(ctx, q, N, Q, Mo, eps_m, eF,
                                                       Rt_qp[..., :N], om[j0:j1], wom[j0:j1], W,
                                                       omp, j0 > 0, sig))
            del W
        E, Z, S = timed(q, "qp", lambda: gw.gw_qp_solve(ctx, p.eps[p.qp], None, eF, omp, sig,
                                                         c.eta, 1e-6, 100))
        out[q] = (E, S)
        torch.cuda.empty_cache()
        log(f"{q}: QP done, status {S.tolist()}")
    # totals per precision: the BF16x3 path's NAF is the FP32 path's
    res = {}
    for q in precs:
        st = dict(times[q])
        for k, val in times[mprec[q]].items():
            if k.startswith("naf_") and q != mprec[q]:
                st[k] = val
        res[q] = {"stage_s": {k: round(val, 3) for k, val in st.items()},
                  "total_s": round(sum(st.values()), 3), "n_naf": n_naf[mprec[q]],
                  "status": out[q][1].tolist()}
    ref = "fp64" if "fp64" in precs else None
    for q in precs:
        if ref and q != ref:
            res[q]["qp_diff_vs_fp64_meV"] = float(np.max(np.abs(out[q][0] - out[ref][0])) *
                                                  HARTREE_MEV)
            if M[q].shape == M[ref].shape:
                # the paths' NAF bases differ by rotations inside near-degenerate
                # eigenspaces, so M^m is compared through invariants of the kept
                # space: its trace and Frobenius norm per Laplace point
                res[q]["chi_invariant_rel_err_vs_fp64"] = max(
                    max(abs(float(torch.trace(M[q][m]) / torch.trace(M[ref][m])) - 1.0),
                        abs(float(torch.linalg.norm(M[q][m]) / torch.linalg.norm(M[ref][m])) - 1.0))
                    for m in range(L))
    line = {"workload": f"{cfg.name}: n_occ={c.n_occ} (n_fc={c.n_fc}), n_virt={v}, "
                        f"n_aux={A}, L={L}, F={F}, Pd={Pd}, Q={Q}, streamed in chunks of "
                        f"{chunk} occupied orbitals",
            "generation_s": round(gen_s, 1), "lt_err_norm": lt_err, "autotune": False,
            "paths": res,
            "eps_qp": {q: out[q][0].tolist() for q in precs}}
    ctx.close()
    del p, M, Rt_qps
    torch.cuda.empty_cache()
    return line


def run_grid_sweep(args, cfg, gw, torch):
    """Fig. 4 on the synthetic workload: G0W0 wall time and the largest QP
    error over the QP states for Laplace grids of L points x modified-GL
    grids of F frequencies, against the FP64 oracle's sum-over-states (no
    Laplace) result on the largest F where it is stored (medium:
    tests/golden/medium_sweep_oracle.json, also giving each SOS row's
    difference from the oracle at its own F), else against this path's own
    sum over states; plus the smallest L whose normalised minimax error is
    below eps_LT = 1e-7 (Sec. 3) on the workload's bounds."""
    import dataclasses
    from gwsynth import make_problem
    prob = make_problem(cfg, dtype=np.float32)
    R = [torch.as_tensor(a).to(device="cuda", dtype=torch.float32).contiguous()
         for a in (prob.R_oo, prob.R_ov, prob.R_qp)]
    ctx = gw.Context(0)
    F_list, L_list = (32, 64, 128), (8, 9, 10, 12, 14, 16, 18)

    def timed(params, reps=2):
        gw.gw_g0w0(ctx, args.prec, params, prob.eps, prob.qp, None, *R)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            E, _, S, _, st = gw.gw_g0w0(ctx, args.prec, params, prob.eps, prob.qp, None, *R)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, E, S, st

    ref_cfg = dataclasses.replace(cfg, n_freq=F_list[-1])
    t_ref, E_ref, S_ref, _ = timed(gw.params_for(ref_cfg, no_lt=True))
    log(f"reference (no Laplace, F={F_list[-1]}): {t_ref * 1e3:.1f} ms")
    gpath = os.path.join(ROOT, "tests", "golden", f"{cfg.name}_sweep_oracle.json")
    oracle = json.load(open(gpath)) if os.path.exists(gpath) else None
    ref_kind = "this path's sum over states"
    if oracle is not None and list(oracle["qp"]) == [int(q) for q in prob.qp]:
        E_ref = np.array(oracle[f"eps_qp_sos_F{F_list[-1]}"])
        ref_kind = "FP64 oracle sum over states"
    log(f"QP errors against the {ref_kind} at F={F_list[-1]}")
    rows = []
    for F in F_list:
        t_sos, E_sos, _, _ = timed(gw.params_for(dataclasses.replace(cfg, n_freq=F), no_lt=True))
        rows.append({"F": F, "L": None, "ms": round(t_sos * 1e3, 2),
                     "speedup": round(t_ref / t_sos, 2),
                     "qp_err_meV": float(np.max(np.abs(E_sos - E_ref)) * HARTREE_MEV)})
        if oracle is not None and f"eps_qp_sos_F{F}" in oracle:
            rows[-1]["vs_oracle_same_F_meV"] = float(
                np.max(np.abs(E_sos - np.array(oracle[f"eps_qp_sos_F{F}"]))) * HARTREE_MEV)
        for L in L_list:
            c2 = dataclasses.replace(cfg, n_freq=F, n_lt=L)
            t, E, S, st = timed(gw.params_for(c2))
            rows.append({"F": F, "L": L, "ms": round(t * 1e3, 2), "speedup": round(t_ref / t, 2),
                         "qp_err_meV": float(np.max(np.abs(E - E_ref)) * HARTREE_MEV),
                         "lt_err_norm": st.lt_err_norm, "status_ok": bool(np.all(S == 0))})
            log(f"F={F} L={L}: {t * 1e3:.1f} ms, QP error {rows[-1]['qp_err_meV']:.3f} meV")
    auto = gw.lt_points_for(prob.eps, cfg, 1e-7)
    print(json.dumps({"grid_sweep": cfg.name, "prec": args.prec, "reference_ms": t_ref * 1e3,
                      "reference": ref_kind, "rows": rows, "auto_L_eps_lt_1e-7": auto}),
          flush=True)
    ctx.close()


def run_batched(args, gw, torch):
    """The batched workload: 64 molecules of uneven size through the batched
    driver (FP32 and BF16x3, a1-a9 after the NAF replayed from a cached
    hipGraph) against per-molecule launches of the single-molecule step
    (FP64 and FP32).  Device-synchronised host times of the second pass of
    each (the first pass autotunes, captures and fills caches); QP energies
    against the per-molecule FP64 path.  Prints its own JSON line."""
    from gwsynth import batched_configs
    from gwsynth.device import make_problem_device
    cfgs = batched_configs()
    t0 = time.perf_counter()
    probs = [make_problem_device(c, device="cuda", dtype=torch.float64) for c in cfgs]
    torch.cuda.synchronize()
    log(f"generated {len(probs)} molecules in {time.perf_counter() - t0:.1f} s")
    ctx = gw.Context(0)
    params = gw.batch_params_for(probs[0].cfg)

    def mols(prec):
        cast = (lambda t: t) if prec == "fp64" else (lambda t: t.to(torch.float32).contiguous())
        return [dict(cfg=p.cfg, eps=p.eps, qp=p.qp, R_oo=cast(p.R_oo), R_ov=cast(p.R_ov),
                     R_qp=cast(p.R_qp)) for p in probs]

    def per_molecule(prec, ms):
        out = []
        for m in ms:
            E, _, S, _, st = gw.gw_g0w0(ctx, prec, gw.params_for(m["cfg"]), m["eps"], m["qp"],
                                        None, m["R_oo"], m["R_ov"], m["R_qp"])
            out.append((E, S))
        return out

    def timed(fn, passes=2):
        res = None
        for k in range(passes):
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
        return dt, res

    m64, m32 = mols("fp64"), mols("fp32")
    t64, r64 = timed(lambda: per_molecule("fp64", m64))
    log(f"per-molecule fp64: {t64:.3f} s")
    t32, r32 = timed(lambda: per_molecule("fp32", m32))
    log(f"per-molecule fp32: {t32:.3f} s")
    out = {"workload": f"batched: {len(probs)} molecules, n_occ in "
                       f"[{min(c.n_occ for c in cfgs)}, {max(c.n_occ for c in cfgs)}], "
                       f"n_virt = 8 n_occ, n_aux = 3 (n_occ + n_virt), NAF kept half, "
                       f"L={params.n_lt}, F={params.n_freq}",
           "per_molecule_fp64_s": t64, "per_molecule_fp32_s": t32}

    def qp_diff(res):
        return float(max(np.max(np.abs(a[0] - b[0])) for a, b in zip(res, r64)) * HARTREE_MEV)

    out["per_molecule_fp32_qp_diff_vs_fp64_meV"] = qp_diff(r32)
    for prec in ("fp32", "bf16x3"):
        tb, (res, stats) = timed(lambda: gw.gw_g0w0_batched(ctx, prec, params, m32, graph=True),
                                 passes=3)
        ok = all(np.all(S == 0) for (_, _, S, _, _) in res)
        out[f"batched_{prec}_graph_s"] = tb
        out[f"batched_{prec}_naf_ms"] = stats.t_naf_ms
        out[f"batched_{prec}_replayed"] = bool(stats.graph_replayed)
        out[f"batched_{prec}_qp_diff_vs_fp64_meV"] = qp_diff([(E, S) for (E, _, S, _, _) in res])
        out[f"batched_{prec}_status_ok"] = ok
        log(f"batched {prec} (graph): {tb:.3f} s, NAF {stats.t_naf_ms:.0f} ms")
        if prec == "fp32":
            # one more pass with kernel timing: the NAF eigensolver's stages
            gw.gw_profile_enable(ctx, True)
            gw.gw_g0w0_batched(ctx, prec, params, m32, graph=True)
            torch.cuda.synchronize()
            parts = {}
            for name in ("naf_eig", "naf_tridiag", "naf_bisect", "naf_invit", "naf_orth",
                         "naf_back"):
                ms, n, _, _ = gw.gw_profile_get(ctx, name)
                parts[name] = round(ms, 2) if n else None
            gw.gw_profile_enable(ctx, False)
            out["batched_naf_stages_ms"] = parts
            log(f"batched NAF stages (ms, summed over molecules): {parts}")
    out["speedup_batched_fp32_vs_per_molecule_fp64"] = t64 / out["batched_fp32_graph_s"]
    out["speedup_batched_fp32_vs_per_molecule_fp32"] = t32 / out["batched_fp32_graph_s"]
    print(json.dumps({"batched": out}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large")
    ap.add_argument("--paper-key", type=int, default=1,
                    help="append one streamed paper-scale FP32 step under 'paper_scale' "
                         "(skipped when --time-limit-s would be exceeded; 0 = off)")
    ap.add_argument("--paper-budget-s", type=float, default=330.0,
                    help="time the paper-scale key is allowed for (generation included)")
    ap.add_argument("--time-limit-s", type=float, default=560.0,
                    help="whole-run limit the paper-scale key must fit in")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="steps of the FP64 path timed for comparison (0 = skip)")
    ap.add_argument("--bf16x3-steps", type=int, default=3,
                    help="steps of the BF16x3 path timed for comparison (0 = skip)")
    ap.add_argument("--evgw-runs", type=int, default=1,
                    help="timed five-cycle evGW runs (Sec. 3, Table 3) after the G0W0 steps "
                         "(0 = skip)")
    ap.add_argument("--no-lt-steps", type=int, default=1,
                    help="steps of the same G0W0 without the Laplace transform (sum over "
                         "states at every frequency, the paper's baseline; 0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--streamed", action="store_true",
                    help="stream the raw tensors in occupied chunks (the paper-scale workload; "
                         "prints its own JSON line)")
    ap.add_argument("--grid-sweep", action="store_true",
                    help="sweep Laplace points x integration frequencies on the workload "
                         "(Fig. 4): time and QP error against the sum-over-states result "
                         "on the largest frequency grid (prints its own JSON line)")
    ap.add_argument("--batched", action="store_true",
                    help="the 64-molecule batched workload: batched driver (FP32, BF16x3; "
                         "graph replay) against per-molecule FP64 / FP32 steps (prints its "
                         "own JSON line)")
    ap.add_argument("--precs", default="fp64,fp32,bf16x3")
    ap.add_argument("--chunk-i", type=int, default=0)
    ap.add_argument("--chunk-gb", type=float, default=12.0)
    ap.add_argument("--screen-gb", type=float, default=60.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the path is built "
              "for one GPU; sharding it over several is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from gwsynth import get_config, make_problem
    from paper_2307_04508_amd import gwlt as gw

    cfg = get_config(args.config)
    if args.streamed:
        t0 = time.perf_counter()
        line = run_streamed(args, cfg, gw, torch)
        line["wall_s"] = round(time.perf_counter() - t0, 1)
        print(json.dumps(line), flush=True)
        return
    if args.grid_sweep:
        run_grid_sweep(args, cfg, gw, torch)
        return
    if args.batched:
        run_batched(args, gw, torch)
        return
    t_start = time.perf_counter()
    t0 = time.perf_counter()
    if cfg.exact_orthonormal:
        import types
        hp = make_problem(cfg)
        prob = types.SimpleNamespace(cfg=cfg, eps=hp.eps, qp=hp.qp,
                                     **{k: torch.as_tensor(getattr(hp, k)).cuda()
                                        for k in ("R_oo", "R_ov", "R_qp")})
    else:
        from gwsynth.device import make_problem_device
        prob = make_problem_device(cfg, device="cuda", dtype=torch.float64,
                                   haar_on_device=cfg.n_aux > 4000)
    torch.cuda.synchronize()
    log(f"generated {cfg.name} inputs on the device in {time.perf_counter() - t0:.1f} s")
    dt = torch.float32 if args.prec == "fp32" else torch.float64

    def upload(dtype):
        return [t.to(dtype=dtype).contiguous() for t in (prob.R_oo, prob.R_ov, prob.R_qp)]

    R = upload(dt)
    ctx = gw.Context(0)
    params = gw.params_for(cfg)

    def step(prec, tens):
        return gw.gw_g0w0(ctx, prec, params, prob.eps, prob.qp, None, *tens)

    for w in range(args.warmup):
        step(args.prec, R)
        log(f"warmup {w + 1}/{args.warmup} done")
    gw.gw_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        E, Z, S, sig, st = step(args.prec, R)
        if (k + 1) % 5 == 0 and k + 1 < args.steps:
            log(f"timed step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = (t1 - t0) / args.steps
    log(f"timed {args.steps} steps: {wall * 1e3:.1f} ms/step, N_NAF={st.n_naf}")
    kname = "chi_syrk_f32" if args.prec == "fp32" else "chi_syrk_f64"
    bname = "bwb_f32" if args.prec == "fp32" else "bwb_f64"
    chi = kernel_rate(gw, ctx, kname)
    bwb = kernel_rate(gw, ctx, bname)
    others = {n: kernel_rate(gw, ctx, n) for n in
              ("naf_syrk", "screen_sweep", "naf_eig", "naf_tridiag", "naf_bisect", "naf_invit",
               "naf_orth", "naf_back", "naf_gemm_f32", "naf_gemm_f64")}
    gw.gw_profile_enable(ctx, False)
    stage_ms = {"naf": st.t_naf_ms, "chi": st.t_chi_ms, "screen": st.t_screen_ms,
                "sigma": st.t_sigma_ms, "qp": st.t_qp_ms, "total": st.t_total_ms}

    peak = PEAK_TFLOPS[args.prec]
    roofline = None
    if chi:
        roofline = {"kernel": kname, "bound": "mfma", "achieved": round(chi["tflops"], 3),
                    "peak": peak, "unit": "TFLOP/s", "frac": round(chi["tflops"] / peak, 4),
                    "traffic": measured_traffic(kname, cfg.name),
                    "avg_ms": round(chi["avg_ms"], 4),
                    "flops_per_launch": chi["flops_per_launch"],
                    "algorithmic_bytes_per_launch": chi["bytes_per_launch"]}

    bf16 = None
    if args.bf16x3_steps > 0 and args.prec == "fp32":
        step("bf16x3", R)
        gw.gw_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.bf16x3_steps):
            Eb, _, Sb, _, _ = step("bf16x3", R)
        torch.cuda.synchronize()
        wb = (time.perf_counter() - t0) / args.bf16x3_steps
        chib = kernel_rate(gw, ctx, "chi_syrk_bf16x3")
        bwbb = kernel_rate(gw, ctx, "bwb_bf16x3")
        splits = {k: kernel_rate(gw, ctx, n) for k, n in (("chi", "chi_split_bf16x3"),
                                                           ("sigma_contraction", "bwb_split_bf16x3"))}
        gw.gw_profile_enable(ctx, False)
        bf16 = {"wall_s": wb, "qp_diff_vs_fp32_meV": float(np.max(np.abs(Eb - E)) * HARTREE_MEV),
                "status": Sb.tolist()}
        for key, kr in (("chi", chib), ("sigma_contraction", bwbb)):
            if kr:
                bf16[key] = {"avg_ms": round(kr["avg_ms"], 4),
                             "tflops_algorithmic": round(kr["tflops"], 3),
                             "frac_of_bf16_peak_executed": round(3 * kr["tflops"] / 2500.0, 4),
                             "frac_of_fp32_peak": round(kr["tflops"] / 157.3, 4)}
                sp = splits[key]
                if sp:
                    # the one-off split of the operands into BF16 hi / lo pairs
                    # (HBM-bound), per step, and the rate with it included
                    per_step = sp["avg_ms"] * sp["launches"] / args.bf16x3_steps
                    mm = kr["avg_ms"] * kr["launches"] / args.bf16x3_steps
                    bf16[key]["split_ms_per_step"] = round(per_step, 4)
                    bf16[key]["split_gbs"] = round(sp["gbs"], 1)
                    bf16[key]["tflops_algorithmic_with_split"] = round(
                        kr["flops_per_launch"] * kr["launches"] / args.bf16x3_steps /
                        ((mm + per_step) * 1e-3) / 1e12, 3)
        log(f"bf16x3 path: {wb * 1e3:.1f} ms/step")

    evgw = None
    if args.evgw_runs > 0:
        gw.gw_evgw(ctx, args.prec, params, 5, prob.eps, prob.qp, None, *R)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.evgw_runs):
            Ee, _, Se, _, ste = gw.gw_evgw(ctx, args.prec, params, 5, prob.eps, prob.qp, None, *R)
        torch.cuda.synchronize()
        evgw = {"cycles": 5, "wall_s": (time.perf_counter() - t0) / args.evgw_runs,
                "naf_ms": round(ste.t_naf_ms, 3), "chi_ms": round(ste.t_chi_ms, 3),
                "screen_ms": round(ste.t_screen_ms, 3), "sigma_ms": round(ste.t_sigma_ms, 3),
                "qp_shift_vs_g0w0_meV": [round(float(x), 3)
                                         for x in (Ee[-1] - Ee[0]) * HARTREE_MEV],
                "last_step_meV": float(np.max(np.abs(Ee[-1] - Ee[-2])) * HARTREE_MEV),
                "status": Se[-1].tolist()}
        log(f"evGW (5 cycles): {evgw['wall_s'] * 1e3:.1f} ms")

    no_lt = None
    if args.no_lt_steps > 0:
        p_sos = gw.params_for(cfg, no_lt=True)
        gw.gw_g0w0(ctx, args.prec, p_sos, prob.eps, prob.qp, None, *R)
        gw.gw_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.no_lt_steps):
            Es, _, Ss, _, sts = gw.gw_g0w0(ctx, args.prec, p_sos, prob.eps, prob.qp, None, *R)
        torch.cuda.synchronize()
        ws = (time.perf_counter() - t0) / args.no_lt_steps
        chis = kernel_rate(gw, ctx, "chi_sos_f32" if args.prec == "fp32" else "chi_sos_f64")
        gw.gw_profile_enable(ctx, False)
        no_lt = {"wall_s": ws, "lt_speedup": ws / wall,
                 "chi_ms": round(sts.t_chi_ms, 3), "chi_speedup_lt": round(sts.t_chi_ms /
                                                                         stage_ms["chi"], 3),
                 "chi_tflops": None if not chis else round(chis["tflops"], 3),
                 "qp_diff_vs_lt_meV": float(np.max(np.abs(Es - E)) * HARTREE_MEV),
                 "status": Ss.tolist()}
        log(f"without the Laplace transform: {ws * 1e3:.1f} ms/step")

    fp64 = None
    if args.fp64_steps > 0 and args.prec != "fp64":
        R64 = upload(torch.float64)
        step("fp64", R64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            E64, _, S64, _, _ = step("fp64", R64)
        torch.cuda.synchronize()
        fp64 = {"wall_s": (time.perf_counter() - t0) / args.fp64_steps,
                "qp_diff_vs_fp32_meV": float(np.max(np.abs(E64 - E)) * HARTREE_MEV)}
        del R64
        log(f"fp64 path: {fp64['wall_s'] * 1e3:.1f} ms/step")

    if args.copy_calibration:
        # one elementwise kernel reading 1 GiB and writing 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB write elementwise kernel done")
        del src, dst

    qp_err = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{cfg.name}_oracle.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        qp_err = {"precision_part_max_meV": float(np.max(np.abs(E - np.array(g["eps_qp_lt"])))
                                                  * HARTREE_MEV),
                  "laplace_part_max_meV": float(np.max(np.abs(np.array(g["eps_qp_lt"]) -
                                                              np.array(g["eps_qp_sos"])))
                                                * HARTREE_MEV),
                  "total_vs_sos_max_meV": float(np.max(np.abs(E - np.array(g["eps_qp_sos"])))
                                                * HARTREE_MEV),
                  "status": S.tolist()}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        cpu = cpu_baseline(prob, torch)
        log(f"oracle: {cpu['measured_s']:.1f} s measured, {cpu['value']:.1f} s extrapolated")

    paper = None
    if args.paper_key and cfg.name != "paper":
        elapsed = time.perf_counter() - t_start
        if elapsed + args.paper_budget_s <= args.time_limit_s:
            del R, prob
            ctx.close()
            ctx = None
            torch.cuda.empty_cache()
            log(f"one streamed paper-scale FP32 step ({elapsed:.0f} s elapsed)")
            t0 = time.perf_counter()
            pargs = argparse.Namespace(**{**vars(args), "precs": "fp32"})
            paper = run_streamed(pargs, get_config("paper"), gw, torch)
            paper["wall_s"] = round(time.perf_counter() - t0, 1)
            log(f"paper scale: {paper['paths']['fp32']['total_s']:.1f} s of stages, "
                f"{paper['wall_s']:.0f} s with generation")
        else:
            paper = {"skipped": f"time budget: {elapsed:.0f} s elapsed + {args.paper_budget_s} s "
                                f"needed > {args.time_limit_s} s"}

    line = {
        "metric": "G0W0 wall s + chi/Sigma TFLOP/s (% MFMA peak), FP32/BF16x3 vs FP64, "
                  "QP err≤1meV",
        "value": wall, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic (seeded)",
        "config": {"workload": f"{cfg.name}: n_occ={cfg.n_occ} (n_fc={cfg.n_fc}), "
                               f"n_virt={cfg.n_virt}, n_aux={cfg.n_aux} -> N_NAF={st.n_naf}, "
                               f"L={cfg.n_lt}, F={cfg.n_freq}, Pd={cfg.n_pade}, Q={cfg.n_qp}",
                   "n_naf": st.n_naf, "precision": args.prec},
        "roofline": roofline,
        "sigma_contraction": None if not bwb else {
            "kernel": bname, "achieved": round(bwb["tflops"], 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(bwb["tflops"] / peak, 4),
            "avg_ms": round(bwb["avg_ms"], 4)},
        "kernels": {k: (None if v is None else {"avg_ms": round(v["avg_ms"], 4),
                                                "launches": v["launches"],
                                                "tflops": round(v["tflops"], 3)})
                    for k, v in others.items()},
        "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()},
        "lt_err_norm": st.lt_err_norm,
        "fp64": fp64,
        "bf16x3": bf16,
        "evgw": evgw,
        "no_laplace": no_lt,
        "qp_err": qp_err,
        "cpu_baseline": cpu,
        "paper_scale": paper,
    }
    print(json.dumps(line), flush=True)
    if ctx is not None:
        ctx.close()


if __name__ == "__main__":
    main()
