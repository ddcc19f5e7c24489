"""Benchmark: Phi + grad Phi target evaluations per second on one MI355X.

One step = one pass of the hot path over the workload: source preparation
(quadrature nodes and folded constants from the device-resident mesh and
sigma; in FMM mode also the octree, expansions and translations) followed by
Phi / grad Phi at every target, all inputs resident in HBM before the timed
region.  Both precisions are timed in the same run; ``value`` is the mixed
path (FP32 pair kernel, FP64 far field / updates) and the FP64 figure is
reported beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2|c5]

Prints ONE JSON line.  The CPU oracle is timed on a bounded target sample of
the same workload (rank 0 only) for the ``cpu_baseline`` field.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Φ+∇Φ target evals/sec, mixed vs FP64 at 1e-6 / 1e-12, 2M-triangle mesh, 1 GPU")
PEAK = {"f64": 78.6, "f32": 157.3}          # TFLOP/s, MI355X published dense vector peaks
FLOP_PER_PAIR = 40.0                        # algorithmic FLOPs per (target, node) pair


def L2P_FLOP(p):
    """Algorithmic FLOPs of a local-expansion evaluation with its gradient at
    one target, order p: about 8 per coefficient."""
    return 8.0 * (p + 1) ** 2
HESS_FLOP_PER_PAIR = 87.0                   # Phi, grad and Hessian of one pair, far form


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest():
    import hashlib
    path = os.path.join(ROOT, "paper_1909_13356_amd", "csrc", "lss_p2p.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary, or None when it was taken on other kernel source or workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = rec.get(kernel)
    if not e or e.get("source_digest") != kernel_digest() or e.get("workload") != workload:
        return None
    return e.get("bytes_per_launch")


def workload(name, scale):
    from workloads import configs
    if name == "c2":
        cfg = configs.config2(n_targets=int(1_000_000 * scale))
        desc = "icosphere level 5 (20480 tri, 245760 Dunavant-6 nodes), sigma 0.05, " \
               "%d targets r~U[0.5,1.5], direct sum" % len(cfg["targets"])
        far = 0
    elif name == "c5":
        cfg = configs.config5(n_targets=int(50_000_000 * scale))
        desc = "graded bumpy sphere (%d tri, %d nodes), sigma_j = D_j/2, %d near-surface targets, octree + FMM" % (
            len(cfg["tris"]), 12 * len(cfg["tris"]), len(cfg["targets"]))
        far = 1
    else:
        raise SystemExit("unknown config " + name)
    return cfg, desc, far


def time_variant(lss, torch, cfg, prec, far, steps, warmup):
    dev = torch.device("cuda")
    v = torch.as_tensor(cfg["verts"], device=dev)
    t = torch.as_tensor(cfg["tris"], device=dev)
    r = torch.as_tensor(cfg["rule"], device=dev)
    s = torch.as_tensor(np.asarray(cfg["sigma"], float), device=dev)
    x = torch.as_tensor(cfg["targets"], device=dev)
    n = x.shape[0]
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    grad = torch.empty((n, 3), dtype=torch.float64, device=dev)
    c = lss.Context(0)
    c.set_sources(v, t, r)
    c.set_sigma(s)
    c.set_options(precision=prec, far_field=far)

    def step():
        c.set_sigma(s)            # invalidates the built state: the step rebuilds it
        c.eval(x, phi=phi, grad=grad)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kms, launches, pairs = 0.0, 0, 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # pair-kernel duration from HIP events on the context stream (last step)
    st = c.stats()
    kms, launches, pairs = st["pair_kernel_ms"], st["pair_kernel_launches"], st["last_pairs"]
    lane_use = st["last_pairs"] / st["lane_pairs"] if st["lane_pairs"] > 0 else None
    tree = {k: st[k] for k in ("n_leaves", "n_boxes", "n_m2l", "tree_depth", "fmm_order")}
    # eval-only timing (built state reused)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        c.eval(x, phi=phi, grad=grad)
    torch.cuda.synchronize()
    el_eval = time.perf_counter() - t1
    # one more evaluation, untimed, whose kernels also count the pairs inside
    # the cut (the method's own near-field work); results are unchanged
    c.set_options(precision=prec, far_field=far, count_useful=1)
    c.eval(x, phi=phi, grad=grad)
    stu = c.stats()
    useful, dipole = stu["useful_pairs"], stu["dipole_pairs"]
    c.close()
    return dict(ms_per_step=1e3 * el / steps, value=n * steps / el, eval_only_per_s=n * steps / el_eval,
                pair_kernel_ms=kms, pair_kernel_launches=launches, pairs_per_step=pairs,
                pairs_per_s=pairs * steps / el, useful_pairs_per_step=useful, useful_pairs_per_s=useful * steps / el,
                dipole_pairs_per_step=dipole,
                n_targets=n, lane_use=lane_use, tree=tree, phi=phi, grad=grad)


def time_newton(lss, torch, cfg, prec, steps, warmup):
    """Chart projection (Newton onto Phi = 1/2) of every chart node of the
    graded surface with the FMM path; one step = build + all iterations."""
    dev = torch.device("cuda")
    v = torch.as_tensor(cfg["verts"], device=dev)
    t = torch.as_tensor(cfg["tris"], device=dev)
    r = torch.as_tensor(cfg["rule"], device=dev)
    s = torch.as_tensor(np.asarray(cfg["sigma"], float), device=dev)
    uv = torch.as_tensor(cfg["chart_uv"], device=dev)
    c = lss.Context(0)
    c.set_sources(v, t, r)
    c.set_sigma(s)
    c.set_options(precision=prec, far_field=lss.FAR_FMM)
    n_nodes = len(cfg["tris"]) * len(cfg["chart_uv"])
    log("bench:   projection")
    for _ in range(warmup):
        c.set_sigma(s)
        c.project(uv, device=True)
    torch.cuda.synchronize()
    el, evals, iters, gms = 0.0, 0, 0, 0.0
    for _ in range(steps):
        c.set_sigma(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, x, st, it = c.project(uv, device=True)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        stt = c.stats()
        evals += stt["last_targets"]
        iters = max(iters, stt["newton_iters"])
        gms += stt["pair_kernel_ms"]
    conv = float((st == 0).sum().item()) / n_nodes
    log("bench:   chart geometry")
    # chart geometry (tangents, area element, normal) at the converged charts:
    # one evaluation of grad Phi at x = T + h H plus the per-node kernel
    c.chart_geometry(uv, h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.chart_geometry(uv, h)
    torch.cuda.synchronize()
    eg = time.perf_counter() - t0
    # degree-8 interpolation of the chart points to 66 new points per triangle
    # (the order-10 lattice), section 3.3
    from workloads import chart_nodes
    log("bench:   chart interpolation")
    ev = torch.as_tensor(chart_nodes(10), device=dev)
    c.chart_interp(uv, x, ev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.chart_interp(uv, x, ev)
    torch.cuda.synchronize()
    ei = time.perf_counter() - t0
    # second derivatives and curvatures of every chart: the Hessian through
    # the octree at x = T + h H plus the per-node kernel (section 3.1)
    log("bench:   chart curvature")
    c.chart_curvature(uv, h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.chart_curvature(uv, h)
    torch.cuda.synchronize()
    ek = time.perf_counter() - t0
    # the paper's target-attached width sigma(x) (lambda 2.5, sigma0 = sqrt(5)
    # max D) at the converged chart points, through the octree: one call
    log("bench:   target-attached sigma(x)")
    c.eval_multiscale(x, 2.5, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.eval_multiscale(x, 2.5, 0.0)
    torch.cuda.synchronize()
    em = time.perf_counter() - t0
    c.close()
    return {"chart_nodes_per_s": n_nodes * steps / el, "target_evals_per_s": evals / el,
            "multiscale_ms": 1e3 * em, "multiscale_points_per_s": n_nodes / em,
            "curvature_nodes_per_s": n_nodes * steps / ek, "curvature_ms": 1e3 * ek / steps,
            "ms_per_step": 1e3 * el / steps, "newton_graph_ms": gms / steps, "iterations": iters,
            "evals_per_node": evals / steps / n_nodes, "converged_frac": conv,
            "geometry_nodes_per_s": n_nodes * steps / eg, "geometry_ms": 1e3 * eg / steps,
            "interp_points_per_s": len(cfg["tris"]) * 66 * steps / ei, "interp_ms": 1e3 * ei / steps}


def time_hessian(lss, torch, steps):
    """Hessian and chart curvature on the 20,480-triangle sphere (sigma 0.05):
    the p = 2 chart nodes (6 per triangle) are projected once; then
    lss_eval_hessian at those points through the octree (FP64 settings) and
    by the direct sum over every pair (the pair rate), lss_chart_curvature
    (octree Hessian plus the per-node second derivatives), and
    lss_eval_multiscale (target-attached sigma(x), direct; pairs counted as
    centroids + nodes)."""
    from workloads import configs, chart_nodes
    c2 = configs.config2(n_targets=1)
    dev = torch.device("cuda")
    uv = torch.as_tensor(chart_nodes(2), device=dev)
    c = lss.Context(0)
    c.set_sources(torch.as_tensor(c2["verts"], device=dev), torch.as_tensor(c2["tris"], device=dev),
                  torch.as_tensor(c2["rule"], device=dev))
    c.set_sigma(np.asarray(c2["sigma"], float))
    c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM)
    h, x, st, it = c.project(uv, device=True)
    n = len(x)
    pairs = n * 12 * len(c2["tris"])
    c.eval_hessian(x)                      # through the octree (near lists + expansions)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.eval_hessian(x)
    torch.cuda.synchronize()
    ef = (time.perf_counter() - t0) / steps
    c.set_options(precision=lss.FP64, far_field=lss.FAR_DIRECT)
    c.eval_hessian(x)                      # every pair
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.eval_hessian(x)
    torch.cuda.synchronize()
    eh = (time.perf_counter() - t0) / steps
    c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM)
    c.chart_curvature(uv, h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.chart_curvature(uv, h)
    torch.cuda.synchronize()
    ec = (time.perf_counter() - t0) / steps
    # the paper's target-attached width sigma(x) (lambda 2.5, sigma0 = sqrt(5) max D)
    # at the same points: a pass over the centroids, then the nodes through
    # the octree (cut widths = the largest sigma_j) or every node
    def timed_ms():
        c.eval_multiscale(x, 2.5, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c.eval_multiscale(x, 2.5, 0.0)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    emf = timed_ms()
    c.set_options(precision=lss.FP64, far_field=lss.FAR_DIRECT)
    em = timed_ms()
    c.close()
    ach = HESS_FLOP_PER_PAIR * pairs / eh / 1e12
    return {"workload": "icosphere, %d tri, %d nodes, sigma 0.05, %d chart nodes (p = 2), FP64 Hessian"
                        % (len(c2["tris"]), 12 * len(c2["tris"]), n),
            "hessian_fmm_ms": 1e3 * ef, "hessian_fmm_points_per_s": n / ef,
            "hessian_ms": 1e3 * eh, "hessian_pairs_per_s": pairs / eh, "hessian_points_per_s": n / eh,
            "hessian_tflops": round(ach, 3), "hessian_frac_f64": round(ach / PEAK["f64"], 4),
            "curvature_ms": 1e3 * ec, "curvature_nodes_per_s": n / ec,
            "multiscale_fmm_ms": 1e3 * emf, "multiscale_fmm_points_per_s": n / emf,
            "multiscale_ms": 1e3 * em, "multiscale_points_per_s": n / em,
            "multiscale_pairs_per_s": n * 13 * len(c2["tris"]) / em}


def time_batch(lss, torch, b, uv, prec, per_surface):
    """One pass over the batch of surfaces: build, Phi / grad Phi at the
    random targets of every surface, Newton projection of every chart node.
    Batched: one context holds all surfaces (one build, one evaluation, one
    projection).  Per surface: the same work surface by surface."""
    dev = torch.device("cuda")
    r = torch.as_tensor(b["rule"], device=dev)
    uvd = torch.as_tensor(uv, device=dev)
    off = b["tri_offsets"]
    if per_surface:
        parts = []
        for m in range(len(off) - 1):
            t0, t1 = off[m], off[m + 1]
            tris = b["tris"][t0:t1]
            v0 = tris.min()
            sel = b["target_mesh"] == m
            parts.append(dict(v=torch.as_tensor(b["verts"][v0:tris.max() + 1], device=dev),
                              t=torch.as_tensor(tris - v0, device=dev),
                              s=torch.as_tensor(b["sigma"][t0:t1], device=dev),
                              x=torch.as_tensor(b["targets"][sel], device=dev)))
    else:
        parts = [dict(v=torch.as_tensor(b["verts"], device=dev), t=torch.as_tensor(b["tris"], device=dev),
                      s=torch.as_tensor(b["sigma"], device=dev), x=torch.as_tensor(b["targets"], device=dev),
                      xm=torch.as_tensor(b["target_mesh"], device=dev),
                      off=torch.as_tensor(b["tri_offsets"], device=dev))]
    ctxs = []
    for q in parts:
        c = lss.Context(0)
        c.set_sources(q["v"], q["t"], r, tri_offsets=q.get("off"))
        c.set_options(precision=prec, far_field=lss.FAR_FMM)
        ctxs.append(c)

    conv = [0, 0]
    hist = torch.zeros(4, dtype=torch.int64, device=dev)

    def step():
        evals = 0
        conv[0] = conv[1] = 0
        hist.zero_()
        for c, q in zip(ctxs, parts):
            c.set_sigma(q["s"])
            c.eval(q["x"], x_mesh=q.get("xm"))
            h, x, st, it = c.project(uvd, device=True)
            evals += q["x"].shape[0] + c.stats()["last_targets"]
            conv[0] += int((st == 0).sum().item())
            conv[1] += st.shape[0]
            hist.add_(torch.bincount(st.to(torch.int64), minlength=4)[:4])
        return evals

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    n_nodes = len(b["tris"]) * len(uv)
    hs = hist.cpu().tolist()
    return {"ms_per_step": 1e3 * el, "target_evals_per_s": evals / el, "chart_nodes_per_s": n_nodes / el,
            "contexts": len(ctxs), "converged_frac": conv[0] / max(conv[1], 1),
            "statuses": {"converged": hs[0], "maxiter": hs[1], "nobracket": hs[2], "degenerate_h": hs[3]}}


def cpu_newton(cfg, n_tris=4):
    """The oracle's Newton projection (FP64 direct sum per evaluation) on the
    chart nodes of a few seeded triangles: about 10 s of CPU work."""
    import oracle
    rng = np.random.default_rng(4321)
    sel = np.sort(rng.choice(len(cfg["tris"]), n_tris, replace=False))
    t0 = time.perf_counter()
    oracle.project(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], cfg["chart_uv"], sel=sel)
    dt = time.perf_counter() - t0
    nn = n_tris * len(cfg["chart_uv"])
    return {"value": nn / dt, "unit": "chart nodes/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d chart nodes of %d triangles (seeded), FP64 direct-sum Newton, %.1f s" % (nn, n_tris, dt)}


def cpu_baseline(cfg, budget_s=15.0, budget1_s=8.0):
    """The oracle (plain FP64 direct sum, no cut, no FMM) on a seeded target
    sample sized to about budget_s of work on every host thread, then on a
    smaller sample on one thread.  Returns the report and, for the error
    report, the sample's indices with the oracle's Phi, grad Phi and the
    condition sums A_Phi = sum |term|."""
    import oracle
    x = cfg["targets"]
    rng = np.random.default_rng(1234)
    nsrc = len(cfg["tris"]) * len(cfg["rule"])
    m = 64
    idx = rng.choice(len(x), m, replace=False)
    t0 = time.perf_counter()
    oracle.evaluate(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], x[idx])
    dt = time.perf_counter() - t0
    m2 = int(min(len(x), max(m, m * budget_s / max(dt, 1e-3))))
    idx = np.sort(rng.choice(len(x), m2, replace=False))
    t0 = time.perf_counter()
    po, go, ao, _ = oracle.evaluate(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], x[idx], with_abs=True)
    dt = time.perf_counter() - t0
    nt = oracle.threads()
    m1 = int(max(1, min(m2, m2 / dt / max(nt, 1) * budget1_s)))
    t0 = time.perf_counter()
    oracle.evaluate(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], x[idx[:m1]], nthreads=1)
    dt1 = time.perf_counter() - t0
    rep = {"value": m2 / dt, "unit": "target evals/s", "cores": nt, "kind": "oracle",
           "sample": "%d of %d targets (seeded), full direct FP64 sum over all %d nodes, %.1f s" % (
               m2, len(x), nsrc, dt),
           "pairs_per_s": m2 * nsrc / dt,
           "single_thread": {"value": m1 / dt1, "unit": "target evals/s", "cores": 1,
                             "pairs_per_s": m1 * nsrc / dt1,
                             "sample": "the first %d targets of the same sample, %.1f s" % (m1, dt1)}}
    return rep, (idx, po, go, ao)


def error_report(phi, grad, ref):
    """Errors of the GPU results at the oracle's sample:
    e_phi = max |dPhi| / max |Phi_oracle|, e_grad likewise with norms;
    pointwise |dPhi| / |Phi_oracle| over targets with |Phi_oracle| >= 1e-3,
    and |dPhi| / A_Phi (A_Phi = sum of |terms|), at median, p99 and max."""
    idx, po, go, ao = ref
    import torch
    ii = torch.as_tensor(idx, device=phi.device)
    p = phi.index_select(0, ii).cpu().numpy()
    g = grad.index_select(0, ii).cpu().numpy()
    dp = np.abs(p - po)
    dg = np.linalg.norm(g - go, axis=1)
    big = np.abs(po) >= 1e-3
    pw = dp[big] / np.abs(po[big])
    ca = dp / ao

    def q(a):
        return {"median": float(np.median(a)), "p99": float(np.quantile(a, 0.99)), "max": float(a.max())} \
            if len(a) else None
    return {"targets": int(len(idx)), "e_phi": float(dp.max() / np.abs(po).max()),
            "e_grad": float(dg.max() / np.linalg.norm(go, axis=1).max()),
            "pointwise_rel_phi": q(pw), "dphi_over_Aphi": q(ca)}


def full_comparison(phi, grad, phi_r, grad_r):
    """The mixed results against the FP64 path's at every target (the FP64
    path matches the oracle's sample to about 1e-14, far below the mixed
    bar): e_phi = max |dPhi| / max |Phi|, e_grad likewise with norms, and
    quantiles of |dPhi| over every 13th target."""
    import torch
    dphi = (phi - phi_r).abs()
    dg = (grad - grad_r).norm(dim=1)
    q = torch.quantile(dphi[::13].double(), torch.tensor([0.5, 0.99, 0.9999], device=dphi.device, dtype=torch.float64))
    return {"targets": int(phi.numel()), "e_phi": float(dphi.max() / phi_r.abs().max()),
            "e_grad": float(dg.max() / grad_r.norm(dim=1).max()),
            "dphi_median": float(q[0]), "dphi_p99": float(q[1]), "dphi_p9999": float(q[2]),
            "targets_above_1e-7": int((dphi > 1e-7 * phi_r.abs().max()).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-newton", action="store_true", help="skip the chart-projection measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-of-surfaces measurement")
    ap.add_argument("--no-hessian", action="store_true", help="skip the Hessian / curvature measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the path is single-GPU; see DESIGN.md "
              "for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1909_13356_amd as lss
    log("bench: building workload", args.config)
    cfg, desc, far = workload(args.config, args.scale)
    log("bench: workload ready:", desc)
    res = {}
    for prec, name in ((lss.FP64, "f64"), (lss.MIXED, "mixed")):
        log("bench: timing", name)
        res[name] = time_variant(lss, torch, cfg, prec, far, args.steps, args.warmup)
        log("bench:", name, json.dumps({k: v for k, v in res[name].items() if k not in ("phi", "grad")}))
    mixed, f64 = res["mixed"], res["f64"]

    def roof(r, dt):
        """Algorithmic FLOPs of one evaluation launch over its duration: 40 per
        pair inside the cut (the near field the method asks for) plus the
        local-expansion evaluation, 8 (p+1)^2 per target; pairs evaluated
        beyond the cut (whole leaves of the near lists) are not counted."""
        # the FP64 evaluation with the default 64-target tiles is k_eval_fmm_f64_split
        kname = ("k_eval_fmm_%s" if far else "k_p2p_direct_%s") % (
            "mixed" if dt == "f32" else ("f64_split" if far else "f64"))
        traffic = measured_traffic(kname, desc)
        if r["pair_kernel_launches"] <= 0 or r["pair_kernel_ms"] <= 0:
            return None
        per_launch = r["pair_kernel_ms"] / r["pair_kernel_launches"] * 1e-3
        p = r["tree"]["fmm_order"]
        l2p = L2P_FLOP(p) * r["n_targets"] if far else 0.0
        useful = r["useful_pairs_per_step"] / r["pair_kernel_launches"]
        ach = (FLOP_PER_PAIR * useful + l2p) / per_launch / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK[dt], "unit": "TFLOP/s",
                "frac": round(ach / PEAK[dt], 4), "traffic": traffic,
                "kernel": kname, "kernel_ms": round(per_launch * 1e3, 4),
                "useful_pairs_per_launch": useful, "flop_per_useful_pair": FLOP_PER_PAIR,
                "l2p_flop_per_target": L2P_FLOP(p) if far else 0.0,
                "executed_pairs_per_launch": r["pairs_per_step"] / r["pair_kernel_launches"],
                "executed_over_useful": round(r["pairs_per_step"] / max(r["useful_pairs_per_step"], 1.0), 3),
                # of the executed pairs, those of the dipole-only loop (nodes beyond the cut of
                # every target of their tile) and the rest, through the full kernel
                "dipole_loop_pairs_per_launch": r["dipole_pairs_per_step"] / r["pair_kernel_launches"],
                "full_kernel_over_useful": round((r["pairs_per_step"] - r["dipole_pairs_per_step"])
                                                 / max(r["useful_pairs_per_step"], 1.0), 3),
                "lane_use": r["lane_use"],
                "executed_tflops": round(FLOP_PER_PAIR * r["pairs_per_step"] / r["pair_kernel_launches"]
                                         / per_launch / 1e12, 3)}

    out = {
        "metric": METRIC, "value": mixed["value"], "unit": "target evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 pair kernel / f64 accumulate+update", "data": "synthetic",
        "config": {"workload": desc},
        "roofline": roof(mixed, "f32"),
        "fp64": {"value": f64["value"], "ms_per_step": f64["ms_per_step"], "roofline": roof(f64, "f64"),
                 "eval_only_per_s": f64["eval_only_per_s"], "pairs_per_s": f64["pairs_per_s"],
                 "useful_pairs_per_s": f64["useful_pairs_per_s"]},
        "mixed": {"eval_only_per_s": mixed["eval_only_per_s"], "pairs_per_s": mixed["pairs_per_s"],
                  "useful_pairs_per_s": mixed["useful_pairs_per_s"]},
    }
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a sample")
        out["cpu_baseline"], ref = cpu_baseline(cfg)
        out["errors"] = {"mixed": error_report(mixed["phi"], mixed["grad"], ref),
                         "f64": error_report(f64["phi"], f64["grad"], ref)}
        out["errors"]["mixed_vs_f64_all_targets"] = full_comparison(mixed["phi"], mixed["grad"], f64["phi"],
                                                                    f64["grad"])
        log("bench: errors", json.dumps(out["errors"]))
    for r in res.values():
        del r["phi"], r["grad"]
    if not args.no_newton:
        from workloads import configs
        del cfg
        c3 = configs.config3()
        nn = len(c3["tris"]) * len(c3["chart_uv"])
        from workloads import triangle_diameters
        dd = triangle_diameters(c3["verts"], c3["tris"])
        newton = {"workload": "graded multiscale torus R=1 r=0.3 with 200 bumps (%d tri, %d nodes, triangle "
                              "diameters graded %.0fx), sigma_j = D_j/2, %d chart nodes (45 per triangle), "
                              "Newton onto Phi = 1/2, octree + FMM" % (
                                  len(c3["tris"]), 12 * len(c3["tris"]), dd.max() / dd.min(), nn)}
        for prec, name in ((lss.FP64, "f64"), (lss.MIXED, "mixed")):
            log("bench: Newton", name)
            newton[name] = time_newton(lss, torch, c3, prec, max(1, min(args.steps, 3)), 1)
            log("bench: Newton", name, json.dumps(newton[name]))
        if not args.no_cpu:
            log("bench: timing the CPU oracle Newton on a sample")
            newton["cpu_baseline"] = cpu_newton(c3)
        out["newton"] = newton
    if not args.no_batch:
        from workloads import configs
        log("bench: building the batch of surfaces")
        c4 = configs.config4()
        b = configs.concat_batch(c4["meshes"])
        b["rule"] = c4["rule"]
        nt, nx = len(b["tris"]), len(b["targets"])
        batch = {"workload": "%d star-shaped surfaces, %d..%d tri each (%d tri, %d nodes), sigma_j = D_j/2, "
                             "%d random targets + %d chart nodes, octree forest + FMM" % (
                                 len(c4["meshes"]), min(len(m["tris"]) for m in c4["meshes"]),
                                 max(len(m["tris"]) for m in c4["meshes"]), nt, 12 * nt, nx, 45 * nt)}
        for prec, name in ((lss.MIXED, "mixed"), (lss.FP64, "f64")):
            log("bench: batch", name)
            batch[name] = time_batch(lss, torch, b, c4["chart_uv"], prec, per_surface=False)
            log("bench: batch", name, json.dumps(batch[name]))
        log("bench: per-surface mixed")
        batch["mixed_per_surface"] = time_batch(lss, torch, b, c4["chart_uv"], lss.MIXED, per_surface=True)
        log("bench: per-surface mixed", json.dumps(batch["mixed_per_surface"]))
        out["batch"] = batch
    if not args.no_hessian:
        log("bench: Hessian and chart curvature")
        out["hessian"] = time_hessian(lss, torch, max(1, min(args.steps, 3)))
        log("bench: Hessian", json.dumps(out["hessian"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
