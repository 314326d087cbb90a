#!/usr/bin/env python3
"""Benchmark: sector-integrand evaluations per second on one MI355X.

One step = one call of sdi_integrate on the batched, uneven workload: 2000
synthetic sectors (4-9 variables, 5-40 terms per factor, up to 3 singular
variables, orders eps^-3..eps^0), a pilot pass of 16 shifts x 2^12 lattice
points per sector, the variance-driven (Neyman) allocation of a 2^31-evaluation
final budget in per-sector lattices of 2^16..2^24 evaluations, and the final
pass in one persistent, graph-captured, autotuned launch, with the compensated
reductions and the combination.  Inputs (compiled sector tables) are resident
on the GPU before timing starts.  The other configurations (the bubble, the
64-sector synthetic set, the Euclidean and the physical double box) are
measured after the headline and reported as extra keys.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6      # MI355X: 256 CUs x 4 SIMD x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
# the headline workload: 2000 sectors, pilot 16 x 2^12 per sector, final budget 2^31
# evaluations in per-sector lattices of 16 x 2^12 .. 16 x 2^20 (2^16 .. 2^24 evaluations)
HEADLINE = dict(shifts=16, seed=1, warmup=0, budget=1 << 31, pilot_log2=12, alloc_min_log2=12, alloc_max_log2=20,
                lattice_log2=12, tile_log2=0, ppt=0)
SYNTH64 = dict(lattice_log2=16, shifts=16, seed=1, warmup=5, warmup_log2=14, nbins=128, tile_log2=0, ppt=0)
KERNEL_SOURCES = ["paper_1511_03614_amd/csrc/eval_real.hpp", "paper_1511_03614_amd/csrc/tiles_real.hpp",
                  "paper_1511_03614_amd/csrc/sdint_internal.h"]
KERNEL_SOURCES_CPLX = KERNEL_SOURCES + ["paper_1511_03614_amd/csrc/eval_cplx.hpp",
                                        "paper_1511_03614_amd/csrc/tiles_cplx.hpp"]


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _bits(e):
    """Multiplies of one exponent under the term encoding (bit 0: x, bit 1: x^2 as x*x, bit 2: x^4 as four x)."""
    return (e & 1) + 2 * ((e >> 1) & 1) + 4 * ((e >> 2) & 1)


def sector_work(sec, order_max: int, pref_lead: int, use_grid: bool, grouped: bool = True):
    """Algorithmic FP64 operations (add/sub/mul/div = 1, FMA = 2) and logarithms per evaluation.

    Counts the arithmetic of the method as the tile kernel performs it: lattice
    tent map and Vegas map; the polynomial terms (a term c prod x_j^e_j costs
    sum e_j multiplies and one add) - with `grouped`, every term once and the
    corner values as sums of the singular-support group sums (one add per
    group and corner it reaches), else every corner's own list; integer powers
    of the factors; the subtraction/series combination for every (corner,
    subset) pair; the monomial and the weighted accumulation.  Logarithms are
    counted apart and not as flops; integer work and compensation (two-sum)
    are not counted.
    """
    import numpy as np
    n = sec.n
    S = [j for j in range(n) if sec.a[j] == -1.0]
    ns = len(S)
    kf = max(0, order_max - pref_lead + ns + 1)
    fl = 2 * n + (6 * n + 2 if use_grid else 0)
    fl += n + 2 * ns
    logs = ns + 1
    fl += sum(abs(int(sec.b[j])) + int(sec.a[j]) for j in range(n) if j not in S) + 3
    if grouped:
        for fac in sec.factors:
            e = fac.exps.astype(np.int64)
            fl += int(sum(_bits(int(v)) for v in e.ravel())) + len(e)
            sup = np.zeros(len(e), dtype=np.int64)
            for i, j in enumerate(S):
                sup |= (e[:, j] != 0).astype(np.int64) << i
            for sg in set(sup.tolist()):
                fl += 1 << (ns - bin(sg).count("1"))
    for W in range(1 << ns):
        zero = [S[i] for i in range(ns) if W >> i & 1]
        for fac in sec.factors:
            if not grouped:
                alive = np.all(fac.exps[:, zero] == 0, axis=1) if zero else np.ones(len(fac.coef), bool)
                e = fac.exps[alive].astype(np.int64)
                fl += int(sum(_bits(int(v)) for v in e.ravel())) + int(alive.sum())
            fl += abs(int(fac.gamma)) + abs(int(fac.delta))
        fl += 4
        logs += 1
        for T in range(1 << ns):
            if T & ~W:
                continue
            nt = bin(T).count("1")
            fl += 1 + 3 * (ns - nt) + 3 * max(0, kf - (ns - nt))
    fl += 3 * kf
    return fl, logs


def sector_work_complex(sec, order_max: int, pref_lead: int, mono_f=None):
    """Algorithmic FP64 operations and transcendentals per evaluation of a
    contour-deformed sector (complex multiply = 6, complex add = 2, real
    coefficient times complex = 2): per corner the gradient and Hessian
    polynomials of the deformation polynomial (real, at the corner point), the
    LDL^T determinant of the n x n complex symmetric Jacobian, the deformed
    point, the factors at complex points, the series of every (corner, subset)
    pair and the accumulation.  Logarithms, atan2, exp and sincos are counted
    apart as transcendentals."""
    import numpy as np
    n = sec.n
    S = [j for j in range(n) if sec.a[j] == -1.0]
    ns = len(S)
    kf = max(0, order_max - pref_lead + ns + 1)
    F = sec.factors[sec.deform_factor]
    fl, tr = 2 * n + n + 2 * ns, 2 * ns + 2 * (n - ns) + 1

    def deriv_terms(exps, coef, j, k=None):
        e = exps.astype(np.int64).copy()
        keep = e[:, j] > 0
        e = e[keep]
        e[:, j] -= 1
        if k is not None:
            keep = e[:, k] > 0
            e = e[keep]
            e[:, k] -= 1
        return e

    for W in range(1 << ns):
        zero = [S[i] for i in range(ns) if W >> i & 1]

        def alive(e):
            return e[np.all(e[:, zero] == 0, axis=1)] if zero and len(e) else e
        # gradient and Hessian polynomials (real), one multiply per exponent bit
        for j in range(n):
            e = alive(deriv_terms(F.exps, F.coef, j))
            fl += int(sum(_bits(int(v)) for v in e.ravel())) + len(e)
            for k in range(j + 1):
                e = alive(deriv_terms(F.exps, F.coef, j, k))
                fl += int(sum(_bits(int(v)) for v in e.ravel())) + len(e) + 4
        fl += 3 * n                                         # sqrt(y(1-y)) arguments, diagonal terms
        tr += n
        for k in range(n):                                  # LDL^T of the complex symmetric matrix
            fl += 6 + 6 + sum(6 + 8 * (i - k) for i in range(k + 1, n))
        fl += 4 * n + 8 * n                                 # deformed point, w_j logs scaled by a_j, b_j
        tr += 3 * n
        for fac in sec.factors:
            e = alive(fac.exps.astype(np.int64))
            fl += int(sum(6 * _bits(int(v)) for v in e.ravel())) + 2 * len(e) + 8
            tr += 3
        fl += 6 + 2
        tr += 3
        for T in range(1 << ns):
            if T & ~W:
                continue
            nt = bin(T).count("1")
            fl += 2 + 2 * (ns - nt) + 10 * max(0, kf - (ns - nt))
    fl += 2 * kf + 2 * kf
    return fl, tr


def launch_work(problem, nevals, lead, use_grid=False, grouped=True):
    """(flops, transcendentals) of one final-pass launch: per-sector work times its
    evaluations; `grouped`: the launch evaluated every term once (sdi_result.grouped)."""
    fl = tr = 0
    for sec, ne in zip(problem.sectors, nevals):
        if problem.complex_mode:
            f, t = sector_work_complex(sec, problem.order_max, lead)
        else:
            f, t = sector_work(sec, problem.order_max, lead, use_grid, grouped)
        fl += f * ne
        tr += t * ne
    return fl, tr


# ------------------------------------------------------------------ CPU baseline (the oracle)

_CPU_PROBLEM = None


def _cpu_init():
    global _CPU_PROBLEM
    import sectorgen
    _CPU_PROBLEM = sectorgen.config4()


def _cpu_task(task):
    """The oracle on one (sector, shift) of 2^m lattice points of the headline
    workload: returns the evaluations, the per-order shift means and mean |w F|."""
    import numpy as np
    from oracle import integrand, integrate, points
    s, r, m, seed = task
    problem = _CPU_PROBLEM
    lead, pref = integrate.prefactor_for(problem)
    sec = problem.sectors[s]
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, r + 1, sec.n, m)[r]
    x, w, _ = points.sector_points(z, m, sh, 0, 1 << m)
    vals, _, _ = integrand.sector_orders(sec, x, problem.order_min, problem.order_max, lead, pref)
    wf = vals * w[None, :]
    q = [integrate.fsum_c(v) / (1 << m) for v in wf]
    return 1 << m, s, r, [[c.real, c.imag] for c in q], np.abs(wf).mean(axis=1).tolist()


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m: int, stride: int, shifts: int = 16, workers: int = 0, seed: int = 1) -> dict:
    """The oracle as it stands on the host's cores: a stratified sample of the
    headline workload (every `stride`-th sector, `shifts` shifts, 2^m lattice
    points: the pilot pass of those sectors) spread over a process pool and
    timed on the wall clock, and the same oracle on one core over the first
    tenth of that sample.  Runs in a process that has not touched the GPU
    (bench.py starts it before its own GPU work).  Also returns the oracle's
    per-shift means of the sample, against which the GPU pass is compared."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import sectorgen
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    workers = workers or max(1, min(16, avail))       # the GPU host grants 16 cores to one GPU's job
    nsec = len(sectorgen.config4().sectors)
    sample = list(range(0, nsec, stride))
    tasks = [(s, r, m, seed) for s in sample for r in range(shifts)]
    _cpu_init()
    t0 = time.perf_counter()
    one = [_cpu_task(t) for t in tasks[: max(1, len(tasks) // 10)]]
    dt1 = time.perf_counter() - t0
    ev1 = sum(o[0] for o in one)
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork"), initializer=_cpu_init) as ex:
        list(ex.map(_cpu_task, [(0, 0, 6, seed)] * workers))      # start every worker before the clock
        t0 = time.perf_counter()
        out = list(ex.map(_cpu_task, tasks, chunksize=2))
        dt = time.perf_counter() - t0
    evals = sum(o[0] for o in out)
    return {"value": evals / dt, "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": f"every {stride}th sector of the 2000 ({len(sample)} sectors) x {shifts} shifts x 2^{m} "
                      f"lattice points ({evals} evals, {dt:.1f} s wall, numpy fp64, {workers} worker processes)",
            "one_core": {"value": ev1 / dt1, "evals": ev1, "s": dt1},
            "nproc": nproc, "affinity": avail, "cpu_model": _cpu_model(),
            "oracle_shift_means": {"m": m, "seed": seed, "shifts": shifts,
                                   "values": [[o[1], o[2], o[3], o[4]] for o in out]}}


def _cpu_baseline_subprocess(m: int, stride: int) -> dict:
    """cpu_baseline in a child interpreter, started before this process uses the GPU."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-log2", str(m),
                        "--cpu-stride", str(stride)], capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"value": None, "error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def traffic_from_profiles(workload: str, sources=None):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if current."""
    for path in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.json")):
        try:
            d = json.load(open(path))
        except (OSError, ValueError):
            continue
        if d.get("kernel_hash") == kernel_hash(sources) and d.get("workload") == workload:
            return d.get("bytes_per_launch")
    return None


def strict_json(v):
    """Non-finite floats become null (strict JSON), recursively."""
    import math
    if isinstance(v, float):
        return v if math.isfinite(v) else None
    if isinstance(v, dict):
        return {k: strict_json(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [strict_json(x) for x in v]
    try:
        import numpy as np
        if isinstance(v, np.generic):
            return strict_json(v.item())
        if isinstance(v, np.ndarray):
            return strict_json(v.tolist())
    except ImportError:
        pass
    return v


def _set(P, ctx, **kw):
    base = dict(lattice_log2=12, shifts=16, seed=1, baker=1, warmup=0, graph=1, sampler=0, budget=0, ppt=0,
                tile_log2=0, pilot_log2=12, alloc_min_log2=12, alloc_max_log2=20, warmup_log2=14, nbins=128,
                small_x=0, slice_log2=0, integrator=0)
    base.update(kw)
    for k, v in base.items():
        P.sdi_set_param(ctx, k, v)


def _err(r):
    """Per-order absolute error (real and imaginary parts combined)."""
    import numpy as np
    return np.hypot(r["err_re"], r["err_im"])


PEAK_BF16_MFMA_TFLOPS = 2500.0   # MI355X dense bf16 matrix peak


def flow_layer_flops(n: int) -> int:
    """Algorithmic flops of one conditioner forward (the three products) summed over the 4 layers."""
    tot = 0
    for l in range(4):
        nb = 1 if n == 1 else len([j for j in range(n) if j % 2 == l % 2])
        na = 0 if n == 1 else n - nb
        tot += 2 * (64 * max(na, 1) + 64 * 64 + 64 * 32 * nb)
    return tot


def equal_time_comparison(P, ctx, name, problem, lambda_max=None, m_pilot=11, share=0.9, max_sel=48,
                          iters=20, batch_log2=11, lr=6e-3, finals=None, plains=None, common=None,
                          select_on="relative", references=None):
    """Error of the learned+batched form against plain batched QMC at equal GPU time.

    Learned form: a plain pilot pass (2^m_pilot lattice points per shift) picks
    the sectors that carry `share` of the pilot's error (select_on = "relative":
    orders weighted by their squared relative error; "top": the highest order
    only, which then also sets the order weights of training and validation;
    at most max_sel sectors); their flows are trained on
    the GPU and validated against the lattice (a flow is kept only where it
    lowers its sector's share of the relative errors and agrees with the
    lattice); then a final pass samples the kept sectors through their flows and
    the rest on the lattice, at each operating point of `finals` (parameter
    sets); its estimate combines, for flow-sampled sectors, the final pass
    with the pilot pass and with a lattice pass over those sectors at the
    final size (`_combine_sectors`).  Its GPU time is pilot + training +
    validation + final pass + that lattice pass.  Plain
    form: lattice passes at each parameter set of `plains`; its error at the
    learned form's time comes from a least-squares power law err = A t^-alpha
    fitted per order to all plain passes (the shift-to-shift error of a
    lattice rule fluctuates from one size to the next, so a fit is steadier
    than interpolating between neighbours; the interpolated value is reported
    as well).
    `common` parameters apply to every pass; `references` (parameter sets) are
    further plain passes reported beside the baseline (e.g. plain QMC with the
    variance-driven allocation, which isolates the flows' share of the gain).
    Device times are the library's own (HIP events on its stream)."""
    import numpy as np
    finals = finals or [dict(lattice_log2=12), dict(lattice_log2=13)]
    plains = plains or [dict(lattice_log2=m) for m in range(10, 17)]
    common = common or {}
    h = P.sdi_problem_create(ctx, problem)

    def run(**kw):
        _set(P, ctx, **{**common, **kw})
        P.sdi_integrate(ctx, h)              # plan, tune and capture once
        return P.sdi_integrate(ctx, h)

    try:
        ns = len(problem.sectors)
        if lambda_max is not None:
            P.sdi_tune_deformation(ctx, h, lambda_max, 4, 10)
        plain = []
        for kw in plains:
            r = run(**kw)
            plain.append((kw, r["ms_total"], _err(r)))
        plain.sort(key=lambda p: p[1])
        refs = []
        for kw in references or []:
            r = run(**kw)
            refs.append({"params": kw, "ms": r["ms_total"], "err": _err(r).tolist()})
        pilot = run(lattice_log2=m_pilot, budget=0)
        pst = _sector_stats(P, ctx, h, ns)
        var = pst[1][:, :, 0] ** 2 + pst[1][:, :, 1] ** 2
        val = pst[0].sum(axis=0)
        scale = np.maximum(np.abs(val) ** 2, var.sum(axis=0))
        if select_on == "top":
            scale[:-1] = np.inf
        w = (var / np.where(scale > 0, scale, 1.0)).sum(axis=1)
        order = np.argsort(-w)
        cum = np.cumsum(w[order]) / max(w.sum(), 1e-300)
        nsel = int(min(max_sel, np.searchsorted(cum, share) + 1, ns))
        sel = sorted(int(s) for s in order[:nsel])
        ow = None
        if select_on == "top":
            ow = np.zeros(problem.norders)
            ow[-1] = 1.0
        P.sdi_flow_init(ctx, h, 1)
        ms_train = P.sdi_flow_train(ctx, h, iters, batch_log2, lr, sectors=sel, order_weights=ow)
        kept, ms_val = P.sdi_flow_validate(ctx, h, m_pilot, order_weights=ow)
        n_kept = [s for s in range(ns) if kept[s]]
        # matrix-core work of the learned sampler: training does, per layer, a
        # recomputed forward and the two backward products (weights and inputs),
        # 3x the forward flops, plus the sampling forward: 4x
        f_train = sum(4 * flow_layer_flops(problem.sectors[s].n) for s in sel) * iters * (1 << batch_log2)
        t = np.array([p[1] for p in plain])
        ep = np.array([p[2] for p in plain])
        lt = np.log(t)
        fit = []                                       # per order: (intercept, slope) in log-log, or None
        for k in range(problem.norders):
            ok = ep[:, k] > 0
            fit.append(np.polyfit(lt[ok], np.log(ep[ok, k]), 1) if ok.sum() >= 2 else None)
        points = []
        for kw in finals:
            fr = run(**kw, sampler=1)
            fst = _sector_stats(P, ctx, h, ns)
            lat, ms_lat = _flow_sector_lattice(P, ctx, problem, kept, {**kw, "seed": 8}, common)
            t_learned = pilot["ms_total"] + ms_train + ms_val + fr["ms_total"] + ms_lat
            pil = ({s: pst[0][s] for s in range(ns)}, {s: pst[1][s] for s in range(ns)})
            fval, ef = _combine_sectors(fst, kept, [pil, lat])
            k = int(np.clip(np.searchsorted(t, t_learned), 1, len(t) - 1))
            a = (np.log(t_learned) - np.log(t[k - 1])) / (np.log(t[k]) - np.log(t[k - 1]))
            with np.errstate(divide="ignore", invalid="ignore"):
                e_int = np.exp((1 - a) * np.log(ep[k - 1]) + a * np.log(ep[k]))
                e_eq = np.array([np.exp(np.polyval(f, np.log(t_learned))) if f is not None else 0.0 for f in fit])
                ratio = np.where(ef > 0, e_eq / ef, np.nan)
            points.append({"final": kw, "ms_total": t_learned, "ms_final_pass": fr["ms_total"],
                           "ms_flow_sampling": fr["ms_warmup"], "err": ef.tolist(),
                           "err_final_pass_alone": _err(fr).tolist(),
                           "value_re": fval.real.tolist(), "value_im": fval.imag.tolist(),
                           "plain_err_at_equal_time": e_eq.tolist(),
                           "plain_err_interpolated": e_int.tolist(),
                           "error_ratio_plain_over_learned": ratio.tolist(),
                           "error_ratio_top_order": float(ratio[problem.norders - 1])})
        return {
            "config": name, "orders": list(range(problem.order_min, problem.order_max + 1)), "sectors": ns,
            "flow_sectors_trained": nsel, "flow_sectors_kept": len(n_kept),
            "pilot": {"lattice_log2": m_pilot, "ms": pilot["ms_total"]},
            "train": {"iters": iters, "batch": 1 << batch_log2, "ms": ms_train,
                      "mfma_bf16_tflops": f_train / (ms_train * 1e-3) / 1e12,
                      "mfma_frac": f_train / (ms_train * 1e-3) / 1e12 / PEAK_BF16_MFMA_TFLOPS},
            "validate_ms": ms_val,
            "learned": points,
            "plain": [{"params": kw, "ms": ms, "err": e.tolist()} for kw, ms, e in plain],
            "plain_fit_loglog": [f.tolist() if f is not None else None for f in fit],
            "plain_references": refs,
            "error_ratio_top_order": [p["error_ratio_top_order"] for p in points],
        }
    finally:
        P.sdi_problem_destroy(h)


def _sector_stats(P, ctx, h, ns):
    """Per-sector means (complex) and standard errors (re, im) of the last pass."""
    import numpy as np
    means, errs = [], []
    for s in range(ns):
        mean, err, _, _ = P.sdi_sector_results(ctx, h, s, 16)
        means.append(mean)
        errs.append(err)
    return np.array(means), np.array(errs)


def _combine_pair(m1, e1, m2, e2):
    """Inverse-variance combination of two independent estimates (complex means,
    errors (re, im)) of the same quantities, real and imaginary parts apart."""
    import numpy as np
    m = np.zeros_like(m1)
    e = np.zeros_like(e1)
    for part, get in ((0, np.real), (1, np.imag)):
        a, b = get(m1), get(m2)
        va, vb = e1[..., part] ** 2, e2[..., part] ** 2
        ok = (va > 0) & (vb > 0)
        w = np.where(ok, vb / np.where(ok, va + vb, 1.0), np.where(vb > 0, 1.0, 0.0))   # weight of the first
        c = w * a + (1 - w) * b
        v = np.where(ok, va * vb / np.where(ok, va + vb, 1.0), np.where(vb > 0, va, vb))
        m = m + (c if part == 0 else 1j * c)
        e[..., part] = np.sqrt(v)
    return m, e


def _combine_sectors(final, kept, extra):
    """The learned form's estimate: a sector sampled by its flow in the final pass
    combines that pass with every further independent estimate of the same
    sector in `extra` (the pilot lattice pass; a lattice pass over the flow
    sectors at the final size), weights 1/sigma^2 per order; the other sectors
    take the final pass alone.  Returns the sum over sectors and its standard
    error per order."""
    import numpy as np
    fm, fe = final
    val = np.zeros(fm.shape[1], dtype=complex)
    var = np.zeros((fm.shape[1], 2))
    for s in range(fm.shape[0]):
        m, e = fm[s], fe[s]
        if kept[s]:
            for xm, xe in extra:
                if s in xm:
                    m, e = _combine_pair(m, e, xm[s], xe[s])
        val += m
        var += e ** 2
    return val, np.sqrt(var[:, 0] + var[:, 1])


def _flow_sector_lattice(P, ctx, problem, kept, params, common):
    """A plain lattice pass over the flow-sampled sectors only (a problem of
    those sectors, so their shifts are drawn independently of the full
    problem's): per-sector means and errors keyed by sector, and its device time."""
    import dataclasses
    import numpy as np
    idx = [s for s in range(len(problem.sectors)) if kept[s]]
    if not idx:
        return ({}, {}), 0.0
    sub = dataclasses.replace(problem, sectors=[problem.sectors[s] for s in idx])
    h = P.sdi_problem_create(ctx, sub)
    try:
        _set(P, ctx, **{**common, **params, "sampler": 0})
        if problem.complex_mode:
            P.sdi_tune_deformation(ctx, h, problem.lam, 4, 10)
        P.sdi_integrate(ctx, h)
        r = P.sdi_integrate(ctx, h)
        m, e = _sector_stats(P, ctx, h, len(idx))
    finally:
        P.sdi_problem_destroy(h)
    return ({s: m[i] for i, s in enumerate(idx)}, {s: e[i] for i, s in enumerate(idx)}), r["ms_total"]


def _learned_pass(P, ctx, h, problem, seed, m_pilot, share, max_sel, iters, batch_log2, lr, final, common):
    """One learned+batched run with the given seed: pilot lattice pass, flows
    for the sectors carrying `share` of the pilot's relative error (at most
    max_sel), GPU training, validation, final mixed pass.  Returns the final
    result and the total device time (pilot + training + validation + final)."""
    import numpy as np
    ns = len(problem.sectors)

    def run(**kw):
        _set(P, ctx, **{**common, "seed": seed, **kw})
        P.sdi_integrate(ctx, h)
        return P.sdi_integrate(ctx, h)

    pilot = run(lattice_log2=m_pilot, budget=0)
    pst = _sector_stats(P, ctx, h, ns)
    var = pst[1][:, :, 0] ** 2 + pst[1][:, :, 1] ** 2
    val = pst[0].sum(axis=0)
    scale = np.maximum(np.abs(val) ** 2, var.sum(axis=0))
    w = (var / np.where(scale > 0, scale, 1.0)).sum(axis=1)
    order = np.argsort(-w)
    cum = np.cumsum(w[order]) / max(w.sum(), 1e-300)
    nsel = int(min(max_sel, np.searchsorted(cum, share) + 1, ns))
    sel = sorted(int(s) for s in order[:nsel])
    P.sdi_flow_init(ctx, h, seed)
    ms_train = P.sdi_flow_train(ctx, h, iters, batch_log2, lr, sectors=sel)
    kept, ms_val = P.sdi_flow_validate(ctx, h, m_pilot)
    fr = run(**final, sampler=1)
    fst = _sector_stats(P, ctx, h, ns)
    lat, ms_lat = _flow_sector_lattice(P, ctx, problem, kept, {**final, "seed": seed + 7}, common)
    pil = ({s: pst[0][s] for s in range(ns)}, {s: pst[1][s] for s in range(ns)})
    value, err = _combine_sectors(fst, kept, [pil, lat])
    return value, err, pilot["ms_total"] + ms_train + ms_val + fr["ms_total"] + ms_lat, int(sum(kept))


def seed_study(P, ctx, name, problem, lambda_max=None, m_pilot=11, share=0.9, max_sel=48, iters=20,
               batch_log2=11, lr=6e-3, final=None, ref=None, plains=None, common=None, seeds=10):
    """Error at equal GPU time against a reference: the learned+batched form and
    plain batched QMC each run with `seeds` independent seeds (shifts, flow
    initialisation and training points); per order, the RMS over seeds of
    |estimate - reference| and of the reported standard error.  The reference is
    one plain lattice run with 256x the points of the learned form's final pass
    (fixed launch shape, no autotuning) and its own seed.  The plain form runs at the two lattice sizes whose device times
    bracket the learned form's mean time; its RMS at that time is interpolated
    in log-log between them."""
    import numpy as np
    final = final or dict(lattice_log2=13)
    ref = ref or dict(lattice_log2=18, shifts=128, tile_log2=14, ppt=1)
    plains = plains or [dict(lattice_log2=m) for m in range(10, 18)]
    common = common or {}
    h = P.sdi_problem_create(ctx, problem)

    def run(seed, **kw):
        _set(P, ctx, **{**common, "seed": seed, **kw})
        P.sdi_integrate(ctx, h)
        return P.sdi_integrate(ctx, h)

    try:
        if lambda_max is not None:
            _set(P, ctx, **{**common, "seed": 1})
            P.sdi_tune_deformation(ctx, h, lambda_max, 4, 10)
        _set(P, ctx, **{**common, "seed": 104729, **ref})
        rr = P.sdi_integrate(ctx, h)
        refv = rr["value"]
        times = [(kw, run(1, **kw)["ms_total"]) for kw in plains]
        times.sort(key=lambda p: p[1])
        est_b, t_b, kept = [], [], []
        for sd in range(1, seeds + 1):
            v, e, t, nk = _learned_pass(P, ctx, h, problem, 1000 + sd, m_pilot, share, max_sel, iters, batch_log2,
                                        lr, final, common)
            est_b.append((v, e))
            t_b.append(t)
            kept.append(nk)
        tb = float(np.mean(t_b))
        ts = np.array([t for _, t in times])
        k = int(np.clip(np.searchsorted(ts, tb), 1, len(ts) - 1))

        def rms(ests):
            d = np.array([np.abs(v - refv) for v, _ in ests])
            e = np.array([e for _, e in ests])
            return np.sqrt((d ** 2).mean(axis=0)), np.sqrt((e ** 2).mean(axis=0))

        ref_var = _err(rr) ** 2

        def corrected(r):
            # |est - ref|^2 averages sigma_est^2 + sigma_ref^2: remove the reference's share
            return np.sqrt(np.maximum(r ** 2 - ref_var, 0.0))

        rb, sb = rms(est_b)
        plain = []
        for kw, t in (times[k - 1], times[k]):
            ests = []
            for sd in range(1, seeds + 1):
                r = run(2000 + sd, **kw)
                ests.append((r["value"], _err(r)))
            ra, sa = rms(ests)
            plain.append({"params": kw, "ms": t, "rms_err": ra.tolist(), "rms_err_ref_corrected": corrected(ra).tolist(),
                          "rms_sigma": sa.tolist()})
        a = (np.log(tb) - np.log(times[k - 1][1])) / (np.log(times[k][1]) - np.log(times[k - 1][1]))
        with np.errstate(divide="ignore", invalid="ignore"):
            r0, r1 = np.array(plain[0]["rms_err"]), np.array(plain[1]["rms_err"])
            r_eq = np.exp((1 - a) * np.log(r0) + a * np.log(r1))
            ratio = np.where(rb > 0, r_eq / rb, np.nan)
            c0, c1 = corrected(r0), corrected(r1)
            c_eq = np.exp((1 - a) * np.log(c0) + a * np.log(c1))
            ratio_c = np.where(corrected(rb) > 0, c_eq / corrected(rb), np.nan)
        return {"config": name, "seeds": seeds,
                "orders": list(range(problem.order_min, problem.order_max + 1)),
                "reference": {"params": ref, "ms": rr["ms_total"], "err": _err(rr).tolist(),
                              "value_re": refv.real.tolist(), "value_im": refv.imag.tolist()},
                "learned": {"final": final, "ms_mean": tb, "flows_kept_mean": float(np.mean(kept)),
                            "rms_err": rb.tolist(), "rms_err_ref_corrected": corrected(rb).tolist(),
                            "rms_sigma": sb.tolist()},
                "plain_bracket": plain,
                "plain_rms_err_at_equal_time": r_eq.tolist(),
                "rms_ratio_plain_over_learned": ratio.tolist(),
                "rms_ratio_ref_corrected": ratio_c.tolist()}
    finally:
        P.sdi_problem_destroy(h)


def cubature_entry(P, ctx, name, problem, maxeval, steps=3, split_frac=0.25, batch_min=1024):
    """The adaptive deterministic cubature (integrator 1) on a workload: the rule
    kernel's rate and roofline (algorithmic flops of the evaluations it made,
    the same per-evaluation count as the lattice kernels' per-corner form),
    the whole call's rate (host bookkeeping of the regions included), regions,
    rounds and error estimates; plain lattice QMC with about as many
    evaluations beside it (16 shifts)."""
    import numpy as np
    ns = len(problem.sectors)
    h = P.sdi_problem_create(ctx, problem)
    try:
        _set(P, ctx, integrator=1)
        for k, v in dict(cub_maxeval=maxeval, cub_epsrel=1e-12, cub_epsabs=0.0, cub_split_frac=split_frac,
                         cub_batch_min=batch_min).items():
            P.sdi_set_param(ctx, k, v)
        P.sdi_integrate(ctx, h)
        runs = [P.sdi_integrate(ctx, h) for _ in range(steps)]
        r = runs[-1]
        nev = [P.sdi_sector_results(ctx, h, s, 16)[3] for s in range(ns)]
        lead = P._prefactor_of(problem)[0]
        fl, _ = launch_work(problem, nev, lead, False, False)
        ms_k = float(np.mean([x["ms_eval_kernel"] for x in runs]))
        ms_t = float(np.mean([x["ms_total"] for x in runs]))
        achieved = fl / (ms_k * 1e-3) / 1e12
        m = max(4, int(round(np.log2(max(1.0, r["n_evals"] / (16.0 * ns))))))
        _set(P, ctx, lattice_log2=m, shifts=16)
        P.sdi_integrate(ctx, h)
        lat = P.sdi_integrate(ctx, h)
        return {"workload": name, "maxeval": maxeval, "evals": int(r["n_evals"]), "regions": int(r["cub_regions"]),
                "rounds": int(r["cub_rounds"]), "ms_rule_kernels": ms_k, "ms_total": ms_t,
                "evals_per_s_kernels": r["n_evals"] / (ms_k * 1e-3), "evals_per_s_total": r["n_evals"] / (ms_t * 1e-3),
                "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
                             "kernel": "k_cubature (all rounds)"},
                "orders": list(range(problem.order_min, problem.order_max + 1)),
                "value_re": r["value"].real.tolist(), "err_estimate": (r["err_re"] + r["err_im"]).tolist(),
                "lattice_same_evals": {"lattice_log2": m, "evals": int(lat["n_evals"]), "ms_total": lat["ms_total"],
                                       "value_re": lat["value"].real.tolist(), "err_re": lat["err_re"].tolist()}}
    finally:
        P.sdi_problem_destroy(h)
        _set(P, ctx)


def adaptive_mc_entry(P, ctx, name, problem, maxeval, steps=3):
    """The sampling adaptive integrators on a workload at the same partition
    budget: integrator 3 (subregion-adaptive Monte Carlo, 1024 points per new
    region) and integrator 4 (partition by spreads with 256 points per new
    region, then a lattice rule of 16 shifts x 2^8 points on every region):
    time in their kernels and per call, regions, evaluations, value and error
    per order."""
    h = P.sdi_problem_create(ctx, problem)
    try:
        out = {"workload": name, "cub_maxeval": maxeval}
        for key, integ, nnew in (("subregion_monte_carlo", 3, 1024), ("partition_then_lattice", 4, 256)):
            _set(P, ctx, integrator=integ, lattice_log2=8, shifts=16)
            for k, v in dict(cub_maxeval=maxeval, cub_epsrel=1e-12, cub_epsabs=0.0, cub_split_frac=0.25,
                             cub_batch_min=1024, suave_nnew=nnew).items():
                P.sdi_set_param(ctx, k, v)
            P.sdi_integrate(ctx, h)
            runs = [P.sdi_integrate(ctx, h) for _ in range(steps)]
            r = runs[-1]
            ms_k = float(sorted(x["ms_eval_kernel"] for x in runs)[steps // 2])
            ms_t = float(sorted(x["ms_total"] for x in runs)[steps // 2])
            out[key] = {"evals": int(r["n_evals"]), "regions": int(r["cub_regions"]), "rounds": int(r["cub_rounds"]),
                        "ms_kernels": ms_k, "ms_total": ms_t, "evals_per_s_kernels": r["n_evals"] / (ms_k * 1e-3),
                        "value_re": r["value"].real.tolist(), "err": _err(r).tolist()}
        return out
    finally:
        P.sdi_problem_destroy(h)
        for k, v in dict(cub_maxeval=1 << 24, cub_epsrel=1e-6, cub_batch_min=1024, suave_nnew=1024).items():
            P.sdi_set_param(ctx, k, v)
        _set(P, ctx)


def monte_carlo_entry(P, ctx, name, problem, m, R=16, warmup=0, steps=3):
    """The Monte Carlo integrator (integrator 2: Philox points, the sampling of
    the paper's default vegasCuba) beside the lattice on the same workload, the
    same evaluations and the same warm-up: final-pass time and error per order."""
    h = P.sdi_problem_create(ctx, problem)
    try:
        out = {"workload": name, "lattice_log2": m, "shifts": R, "warmup": warmup}
        for key, integ in (("lattice", 0), ("monte_carlo", 2)):
            _set(P, ctx, lattice_log2=m, shifts=R, warmup=warmup, integrator=integ)
            P.sdi_integrate(ctx, h)
            runs = [P.sdi_integrate(ctx, h) for _ in range(steps)]
            r = runs[-1]
            out[key] = {"evals": int(r["n_evals"]), "ms_eval_kernel": float(sorted(x["ms_eval_kernel"] for x in runs)[steps // 2]),
                        "value_re": r["value"].real.tolist(), "err": _err(r).tolist()}
        e_l, e_m = out["lattice"]["err"], out["monte_carlo"]["err"]
        out["error_ratio_mc_over_lattice"] = [b / a if a > 0 else None for a, b in zip(e_l, e_m)]
        return out
    finally:
        P.sdi_problem_destroy(h)
        _set(P, ctx)


def text_integrand_rate(P, ctx, steps: int = 5):
    """Throughput of the text path (sdi_problem_from_text) on an integrand of the
    size class the paper's database holds (~200 KB of text): 3000 signed terms of
    nested powers, logs and quotients over 6 variables, 8 intermediate functions;
    16 shifts x 2^14 lattice points per pass."""
    from sectorgen import textgen
    text = textgen.random_text(999, 6, nfuncs=8, depth=3, terms=3000)
    for k, v in dict(lattice_log2=14, shifts=16, seed=1, warmup=0, sampler=0, budget=0, tile_log2=0, ppt=0).items():
        P.sdi_set_param(ctx, k, v)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        P.sdi_integrate(ctx, h)
        ms = []
        for _ in range(steps):
            r = P.sdi_integrate(ctx, h)
            ms.append(r["ms_eval_kernel"])
    finally:
        P.sdi_problem_destroy(h)
    ms_k = sorted(ms)[len(ms) // 2]
    return {"text_bytes": len(text), "vars": 6, "evals_per_pass": int(r["n_evals"]),
            "ms_kernel_median": ms_k, "evals_per_s": r["n_evals"] / (ms_k * 1e-3),
            "tile_log2": r["tile_log2"], "blocks": r["blocks"]}


def endpoint_precision_cost(P, ctx, problem, steps: int = 5):
    """Final-pass kernel time of the 64-sector synthetic workload with the
    endpoint-precision mode (points closer to a singular face than small_x
    evaluated in double-double) against the fp64 pass, median of `steps`
    passes each."""
    _set(P, ctx, **SYNTH64)
    h = P.sdi_problem_create(ctx, problem)
    res = {}
    try:
        for sx in (0, 1e-3, 1e-2):
            P.sdi_set_param(ctx, "small_x", sx)
            P.sdi_integrate(ctx, h)
            ms = sorted(P.sdi_integrate(ctx, h)["ms_eval_kernel"] for _ in range(steps))
            res[str(sx)] = ms[len(ms) // 2]
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
    return {"ms_final_pass": res, "ratio_1e-3": res["0.001"] / res["0"], "ratio_1e-2": res["0.01"] / res["0"]}


def measure(P, ctx, problem, params, steps, warmup, lambda_max=None, conservative_if_imf=False):
    """Steps of sdi_integrate on one workload: wall time per step (the clock
    bracketed by device synchronisations), device and final-pass kernel times
    (HIP events on the library's stream), per-sector final evaluations."""
    import numpy as np
    import torch
    _set(P, ctx, **params)
    h = P.sdi_problem_create(ctx, problem)
    try:
        tuned = None
        if lambda_max is not None:
            tuned = {"lambda": P.sdi_tune_deformation(ctx, h, lambda_max, 4, 10).tolist(), "conservative": False}
            r = P.sdi_integrate(ctx, h)
            if conservative_if_imf and r["n_imf_positive"] > 0:
                tuned = {"lambda": P.sdi_tune_deformation(ctx, h, lambda_max, 4, 10, conservative=True).tolist(),
                         "conservative": True, "imf_positive_before": int(r["n_imf_positive"])}
        for _ in range(warmup):
            r = P.sdi_integrate(ctx, h)
        torch.cuda.synchronize()
        kms, pms, dms, evals = [], [], [], 0
        t0 = time.perf_counter()
        for _ in range(steps):
            r = P.sdi_integrate(ctx, h)
            kms.append(r["ms_eval_kernel"])
            pms.append(r["ms_pilot_kernel"])
            dms.append(r["ms_total"])
            evals += r["n_evals"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ns = len(problem.sectors)
        R = params.get("shifts", 16)
        nev = [P.sdi_sector_results(ctx, h, s, R)[3] for s in range(ns)]
        return {"r": r, "evals_per_step": evals // steps, "wall_s": dt, "ms_per_step": dt / steps * 1e3,
                "value": evals / dt, "ms_kernel": float(np.mean(kms)), "ms_device": float(np.mean(dms)),
                "ms_pilot_kernel": float(np.mean(pms)), "pilot_log2": params.get("pilot_log2", 12)
                if params.get("budget", 0) else None, "nevals": nev, "tuned": tuned, "steps": steps}
    finally:
        P.sdi_problem_destroy(h)


def roofline(P, problem, m, kernel, workload, use_grid=False, sources=None):
    """Achieved FP64 rate of the dominant kernel, the final-pass tile kernel.
    Under budget allocation the pilot pass launches it too; where both ran the
    same instance (sdi_result.pilot_same_kernel) the figures cover both
    launches of a step (mean flops and duration per launch, as a profiler's
    per-kernel average sees them), else the final pass alone."""
    lead = P._prefactor_of(problem)[0]
    r = m["r"]
    grouped = bool(r["grouped"])
    fl, tr = launch_work(problem, m["nevals"], lead, use_grid, grouped)
    ms, launches, note = m["ms_kernel"], 1, "final pass"
    if m.get("pilot_log2") is not None and r["pilot_same_kernel"]:
        R = 16
        pf, pt = launch_work(problem, [R << m["pilot_log2"]] * len(problem.sectors), lead, use_grid, grouped)
        fl, tr, ms, launches = fl + pf, tr + pt, ms + m["ms_pilot_kernel"], 2
        note = "pilot and final pass (same instance), per launch"
    achieved = fl / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": traffic_from_profiles(workload, sources),
            "kernel": kernel, "launches": note, "ms_per_launch": ms / launches, "flops_per_launch": fl / launches,
            "ms_final_pass": m["ms_kernel"], "transcendentals_per_s": tr / (ms * 1e-3)}


def _kernel_name(r, problem, nvmax, nsm):
    """Template arguments of the final-pass instance the run used (sdi_result:
    points per thread, waves, grouped or per-corner term lists)."""
    if problem.complex_mode:
        return f"k_tiles_cplx<{nvmax}, {r['ppt']}, KM, 0, {r['waves_per_simd']}> (final pass)"
    if r["grouped"]:
        return f"k_tiles_real<{nvmax}, {r['ppt']}, KM, 0, {r['waves_per_simd']}, {nsm}, false, 2> (final pass)"
    return f"k_tiles_real<{nvmax}, {r['ppt']}, KM, 0, {r['waves_per_simd']}> (final pass, per-corner term lists)"


def _classes(problem):
    """Register class and singular-variable bound of the final pass instances."""
    nv = max(s.n for s in problem.sectors)
    nsm = max(int(sum(s.a == -1.0)) for s in problem.sectors)
    nvc = 4 if nv <= 4 else 6 if nv <= 6 else 8 if nv <= 8 else 10 if nv <= 10 else 16
    return nvc, (2 if nsm <= 2 else nsm)


def config_entry(P, problem, m, workload, use_grid=False, sources=None):
    nvc, nsm = _classes(problem)
    r = m["r"]
    return {"evals_per_s": m["value"], "ms_per_step": m["ms_per_step"], "evals_per_step": m["evals_per_step"],
            "steps": m["steps"], "ms_device_per_step": m["ms_device"],
            "final_evals": int(sum(m["nevals"])), "points_per_thread": r["ppt"], "waves_per_simd": r["waves_per_simd"],
            "tile_log2": r["tile_log2"], "blocks": r["blocks"], "n_nonfinite": int(r["n_nonfinite"]),
            "n_imf_positive": int(r["n_imf_positive"]), "deformation": m["tuned"],
            "roofline": roofline(P, problem, m, _kernel_name(r, problem, nvc, nsm), workload, use_grid, sources),
            "result": {"orders": list(range(problem.order_min, problem.order_max + 1)),
                       "value_re": r["value"].real.tolist(), "value_im": r["value"].imag.tolist(),
                       "err_re": r["err_re"].tolist(), "err_im": r["err_im"].tolist()}}


def parity_vs_oracle(P, ctx, problem, cpu):
    """Per-coefficient error of the GPU against the oracle on identical points:
    a plain pass (the pilot's lattice size, seed and shifts) over all sectors,
    compared shift by shift with the oracle's means of the CPU sample (computed
    by the cpu_baseline leg).  Per order: the largest |gpu - oracle| relative to
    max(|oracle|, mean |w F|) over the sample's (sector, shift) means, and the
    relative error of the sample's total."""
    import numpy as np
    om = cpu.get("oracle_shift_means") if cpu else None
    if not om:
        return None
    R = om["shifts"]
    _set(P, ctx, lattice_log2=om["m"], shifts=R, seed=om["seed"])
    h = P.sdi_problem_create(ctx, problem)
    try:
        P.sdi_integrate(ctx, h)
        K = problem.norders
        worst = np.zeros(K)
        tot_g = np.zeros(K, complex)
        tot_o = np.zeros(K, complex)
        cache = {}
        for s, r, q, scale in om["values"]:
            if s not in cache:
                cache[s] = P.sdi_sector_results(ctx, h, s, R)[2]
            g = cache[s][r]
            o = np.array([complex(a, b) for a, b in q])
            d = np.abs(g - o) / np.maximum(np.maximum(np.abs(o), np.array(scale)), 1e-300)
            worst = np.maximum(worst, d)
            tot_g += g
            tot_o += o
        return {"orders": list(range(problem.order_min, problem.order_max + 1)),
                "max_rel_err_per_shift_mean": worst.tolist(),
                "rel_err_of_sample_total": (np.abs(tot_g - tot_o) / np.abs(tot_o)).tolist(),
                "compared": f"{len(om['values'])} (sector, shift) means, 2^{om['m']} points each"}
    finally:
        P.sdi_problem_destroy(h)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-log2", type=int, default=12)
    ap.add_argument("--cpu-stride", type=int, default=10)
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--tune-load", default=None,
                    help="load autotuner decisions (sdi_tune_load) before the run, so profiles time the same instance")
    ap.add_argument("--tune-save", default=None, help="save the autotuner decisions of the run (sdi_tune_save)")
    ap.add_argument("--only", default=None,
                    help="profiling aid: run only this workload (batched2000, synthetic64, bubble, doublebox, "
                         "doublebox_physical, adaptive_mc: the sampling adaptive integrators) and print its entry")
    ap.add_argument("--no-equal-time", action="store_true",
                    help="skip the learned-sampler comparison (double box, Euclidean and physical)")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="profiling aid: three device-to-device copies of 256 MiB (the reference that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters to bytes), then exit")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_log2, args.cpu_stride)), flush=True)
        return 0
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py: this benchmark measures one GPU only (asked for --gpus {args.gpus}); "
              "sectors would shard across GPUs by longest-processing-time assignment, but no multi-GPU run is made.",
              file=sys.stderr)
        return 2
    # the oracle's CPU rate first, in a child process, before anything here touches the GPU
    cpu = None if (args.no_cpu_baseline or args.only) else _cpu_baseline_subprocess(args.cpu_log2, args.cpu_stride)
    import torch  # noqa: F401
    import paper_1511_03614_amd as P
    import sectorgen
    from sectorgen.feynman import double_box_problem

    ctx = P.sdi_ctx_create(0)
    if args.tune_load:
        P.sdi_tune_load(ctx, args.tune_load)
    workloads = {
        "batched2000": lambda: (sectorgen.config4(), HEADLINE, {}),
        "synthetic64": lambda: (sectorgen.config2(), SYNTH64, {}),
        "bubble": lambda: (sectorgen.config1(), dict(lattice_log2=13, shifts=8, seed=1), {}),
        "doublebox": lambda: (double_box_problem(-3.0, -1.0, 0.0, order_max=0),
                              dict(shifts=16, seed=1, budget=100_000_000, pilot_log2=10, alloc_min_log2=10,
                                   alloc_max_log2=18), {}),
        "doublebox_physical": lambda: (double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5),
                                       dict(lattice_log2=16, shifts=16, seed=1),
                                       dict(lambda_max=0.5, conservative_if_imf=True)),
    }
    if args.only == "adaptive_mc":
        ent = adaptive_mc_entry(P, ctx, "synthetic64", sectorgen.config2(), 1 << 22)
        P.sdi_ctx_destroy(ctx)
        print(json.dumps(strict_json(ent), allow_nan=False), flush=True)
        return 0
    if args.only:
        prob, prm, kw = workloads[args.only]()
        m = measure(P, ctx, prob, prm, args.steps, args.warmup, **kw)
        ent = config_entry(P, prob, m, args.only, use_grid=prm.get("warmup", 0) > 0,
                           sources=KERNEL_SOURCES_CPLX if prob.complex_mode else None)
        if args.tune_save:
            P.sdi_tune_save(ctx, args.tune_save)
        P.sdi_ctx_destroy(ctx)
        print(json.dumps(strict_json({"workload": args.only, **ent}), allow_nan=False), flush=True)
        return 0
    problem = sectorgen.config4()
    m = measure(P, ctx, problem, HEADLINE, args.steps, args.warmup)
    head = config_entry(P, problem, m, "batched2000")
    r = m["r"]
    out = {
        "metric": "sector-integrand evals/s (FP64) + error vs plain QMC at equal GPU time",
        "value": m["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched2000: 2000 synthetic sectors, 4-9 variables, 5-40 terms per factor, |S| <= 3, "
                               "orders eps^-3..eps^0; per step a pilot pass of 16 shifts x 2^12 lattice points per "
                               "sector, Neyman allocation of a 2^31-evaluation final budget in per-sector lattices of "
                               "2^16..2^24 evaluations, one persistent graph-captured autotuned final launch",
                   "evals_per_step": m["evals_per_step"], "final_evals_per_step": head["final_evals"],
                   "points_per_thread": r["ppt"], "waves_per_simd": r["waves_per_simd"],
                   "tile_log2": r["tile_log2"], "blocks": r["blocks"]},
        "roofline": head["roofline"],
        "result": head["result"],
        "n_nonfinite": head["n_nonfinite"],
    }
    if args.tune_save:
        P.sdi_tune_save(ctx, args.tune_save)
    out["parity_vs_oracle"] = parity_vs_oracle(P, ctx, problem, cpu)
    if not args.no_extras:
        extra = {}
        for name in ("synthetic64", "bubble", "doublebox", "doublebox_physical"):
            prob, prm, kw = workloads[name]()
            steps = 50 if name == "bubble" else 5
            mm = measure(P, ctx, prob, prm, steps, 2, **kw)
            extra[name] = config_entry(P, prob, mm, name, use_grid=prm.get("warmup", 0) > 0,
                                       sources=KERNEL_SOURCES_CPLX if prob.complex_mode else None)
        extra["bubble"]["note"] = "latency-dominated (2 sectors, 1 variable): ms_per_step is the figure, not evals/s"
        out["configs"] = extra
        out["text_integrand"] = text_integrand_rate(P, ctx)
        out["cubature"] = [cubature_entry(P, ctx, "synthetic64", sectorgen.config2(), 1 << 24),
                           cubature_entry(P, ctx, "doublebox (Euclidean, 282 sectors)",
                                          double_box_problem(-3.0, -1.0, 0.0, order_max=0), 1 << 24)]
        out["endpoint_precision"] = endpoint_precision_cost(P, ctx, sectorgen.config2())
        out["monte_carlo"] = monte_carlo_entry(P, ctx, "synthetic64, 5 Vegas warm-up iterations", sectorgen.config2(),
                                               16, warmup=5)
        out["adaptive_monte_carlo"] = adaptive_mc_entry(P, ctx, "synthetic64", sectorgen.config2(), 1 << 22)
    if not args.no_equal_time:
        lat = [dict(lattice_log2=m) for m in range(10, 17)]
        alloc = dict(pilot_log2=10, alloc_min_log2=12, alloc_max_log2=20)
        out["error_vs_plain_qmc"] = [
            equal_time_comparison(P, ctx, "double box, s=-3, t=-1, massless (Euclidean, 282 sectors, eps^-4..eps^0)",
                                  double_box_problem(-3.0, -1.0, 0.0, order_max=0), plains=lat,
                                  finals=[dict(lattice_log2=m) for m in (12, 13, 14)]),
            equal_time_comparison(P, ctx, "batched2000: 2000 synthetic sectors, 4-9 variables, 5-40 terms, "
                                          "eps^-3..eps^0; both forms with per-sector budgets 2^16..2^24 by "
                                          "Neyman allocation",
                                  sectorgen.config4(), m_pilot=10, max_sel=64, common=alloc,
                                  plains=[dict(budget=1 << b) for b in range(26, 32)],
                                  finals=[dict(budget=1 << b) for b in (28, 29, 30)]),
            equal_time_comparison(P, ctx, "double box, s=5, t=-2, m^2=1 (physical, contour deformation, "
                                          "lambda tuned in (0, 0.5], 30 sectors, eps^-4..eps^0)",
                                  double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5),
                                  lambda_max=0.5, plains=lat, finals=[dict(lattice_log2=m) for m in (12, 13, 14)]),
        ]
        out["error_rms_over_seeds"] = [
            seed_study(P, ctx, "double box, s=-3, t=-1, massless (Euclidean, 282 sectors)",
                       double_box_problem(-3.0, -1.0, 0.0, order_max=0)),
            seed_study(P, ctx, "double box, s=5, t=-2, m^2=1 (physical, 30 sectors, lambda tuned in (0, 0.5])",
                       double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5), lambda_max=0.5),
        ]
    P.sdi_ctx_destroy(ctx)
    if cpu is not None:
        cpu = dict(cpu)
        cpu.pop("oracle_shift_means", None)
        out["cpu_baseline"] = cpu
    print(json.dumps(strict_json(out), allow_nan=False), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
