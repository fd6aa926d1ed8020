"""Benchmark: matrix-free isogeometric K-L solves on one MI355X.

One step = the full hot path on the largest single-GPU workload: the unit
cube with p = 2 and 64^3 elements (N = 287,496 unknowns; a dense FP64 A
would take 661 GB), Gaussian kernel ell = 0.2, M = 200 eigenpairs, block
b = 64, Galerkin-IBQ, FP32 kernel tiles and FP32 MFMA contraction: one
complete K-L solve (block Krylov eigensolver on the device around the
matrix-free operator: Kronecker transfers, the fused on-the-fly kernel
product of 287,496^2 pairs per block, FP64 Kronecker solves).

Printed: one JSON line.  value = kernel-pair evaluations per second over the
whole timed region (all steps, eigensolver included), with K-L solves/s,
per-solve latency percentiles, the eigenvalue error against the stored exact
FP64 product-of-1D spectrum (tests/golden/cube_p2_64_reference_spectra.json),
the roofline of the fused kernel product (device time from HIP events on its
launch stream), a second pass in split-BF16 precision, a short serving leg
(128 requests of the serving stream at 1.5x the one-at-a-time service rate,
continuous batching against one-at-a-time solves) and the FP64 CPU oracle
timed on a bounded sample of the same kernel product.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Γ-pair evals/s vs roofline; K-L solves/s + p99 latency @1e-6 eig err"

# MI355X unit counts: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 39.32e12
# lane-instructions/s of non-packed FP32 VALU work; v_exp_f32 issues at half
# rate (two issue slots).  Gaussian pair in the centred Gram form, which the
# kernel takes for row blocks of small extent (every workload here): the
# distance comes from the matrix cores, the VALU keeps the exp = 2 slots (the
# difference form, for wide row blocks, takes 3 sub + mul + 2 fma + exp = 8).
# Exponential pair: 3 sub + 2 add (abs as operand modifiers) + exp = 7 slots.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
SLOTS = {"gaussian": 2, "exponential": 7}
# The contraction: b/16 v_mfma_f32_16x16x4_f32 (2048 flops each) per 64 pairs,
# published dense FP32 matrix peak 157.3 TFLOP/s; the Gram form adds one more
# per 256 pairs for the distances.  On gfx950 FP32 MFMA and VALU work do not
# overlap (measured: mixed waves take the sum of the two times), so the
# attainable rate of the FP32 path is the serial combination of both.
MFMA_F32_FLOPS = 157.3e12
MFMA_BF16_FLOPS = 2.5e15   # published dense BF16 matrix peak


def mfma_per_64_pairs(kernel, b):
    return b / 16.0 + (0.25 if kernel == "gaussian" else 0.0)


def mfma_pairs(b):
    """FP32 matrix-core bound of the contraction: 2 b flops per pair."""
    return MFMA_F32_FLOPS / (2.0 * b)


def serial_peak_pairs(kernel, b):
    mfma_issue_pairs = MFMA_F32_FLOPS / 2048.0 * 64.0 / mfma_per_64_pairs(kernel, b)
    return 1.0 / (1.0 / peak_pairs(kernel) + 1.0 / mfma_issue_pairs)


def peak_pairs(kernel):
    return VALU_SLOTS_PER_S / SLOTS[kernel]


# HBM traffic of the FP32 kernel product per launch: rocprofv3 --pmc
# FETCH_SIZE, then WRITE_SIZE, averaged over the product's launches in a run
# of this workload, each scaled by what the same counter reads for a plain
# 256 MiB device copy (FETCH x 2.0, WRITE x 1.0); the profiles under profiles/
# hold the runs.  Valid only for the kernel source it was measured on.
# Algorithmic bytes per launch: every point's coordinates (16 B), Y row
# (4 b B) and Z row (4 b B) once, plus the row and column scales.
TRAFFIC = {
    "cube20": {"gamma_src_sha256_16": "e9865e3b896f266a", "fetch_bytes": 36.85e6, "write_bytes": 54.48e6,
               "algorithmic_bytes": 33.9e6},
    "cube64": {"gamma_src_sha256_16": "e9865e3b896f266a", "fetch_bytes": 5.919e9, "write_bytes": 7.360e7,
               "algorithmic_bytes": 287496 * (2 * 16 + 8 * 64 + 4)},
}


def measured_traffic(name):
    import hashlib
    t = TRAFFIC[name]
    src = os.path.join(ROOT, "paper_2101_00629_amd", "csrc", "gamma.hip")
    with open(src, "rb") as f:
        if t["gamma_src_sha256_16"] is None or hashlib.sha256(f.read()).hexdigest()[:16] != t["gamma_src_sha256_16"]:
            return None
    return t["fetch_bytes"] + t["write_bytes"]


WORKLOADS = {
    "cube64": "unit cube p=2 64^3 (N=287496), Gaussian l=0.2, M=200, b=64, Galerkin-IBQ: one full K-L solve "
              "(287496^2 kernel pairs per block product)",
    "cube20": "unit cube p=3 20^3 (N=12167), M=50, b=16: Galerkin-IBQ + collocation x Gaussian(l=0.5) + "
              "exponential-L1(l=1), one full K-L solve each",
}


def workload(name, precision="fp32"):
    from workloads import cube_p2_64, cube_p3_20
    if name == "cube64":
        return [cube_p2_64("galerkin", precision=precision)]
    probs = []
    for method in ("galerkin", "collocation"):
        for kernel in ("gaussian", "exponential"):
            probs.append(cube_p3_20(method, kernel, precision=precision))
    return probs


GOLDEN = {"cube64": os.path.join(ROOT, "tests", "golden", "cube_p2_64_reference_spectra.json"),
          "cube20": os.path.join(ROOT, "tests", "golden", "cube_p3_20_reference_spectra.json")}


def reference_spectrum(name, p):
    """Stored FP64 reference (tests/golden/make_cube_p2_64_reference.py and
    tests/golden/make_cube_reference.py write them from the oracle)."""
    with open(GOLDEN[name]) as f:
        return np.array(json.load(f)["spectra"][f"{p['method']}-{p['kernel']}"]["lambda"])[:p["M"]]


def floored_rel_errors(ref, lam, tau=1e-2):
    """|lam - ref| / max(|ref|, tau |ref_1|)."""
    ref, lam = np.asarray(ref), np.asarray(lam)[:len(ref)]
    return np.abs(lam - ref) / np.maximum(np.abs(ref), tau * abs(ref[0]))


def cpu_baseline(probs, seconds_target=20.0):
    """FP64 C/OpenMP oracle kernel product on row samples of each problem."""
    from oracle import cmatvec, collocation, galerkin
    total_pairs, total_time = 0.0, 0.0
    rng = np.random.default_rng(5)
    per = seconds_target / len(probs)
    parts = []
    # calibrate the rate on a small slice first
    for p in probs:
        if p["method"] == "galerkin":
            o = galerkin.GalerkinIBQ("cube", p["p"], p["nel"], p["kernel"], p["ell"])
            Xr, Xc = o.X, o.X
        else:
            o = collocation.Collocation("cube", p["p"], p["nel"], p["kernel"], p["ell"])
            Xr, Xc = o.Xc, o.Xq
        Y = rng.standard_normal((len(Xc), p["block"]))
        nprobe = 256
        t0 = time.perf_counter()
        cmatvec.gamma_apply(p["kernel"], 1.0, p["ell"], Xr[:nprobe], Xc, Y)
        rate = nprobe * len(Xc) / max(time.perf_counter() - t0, 1e-6)
        rows = int(min(len(Xr), max(64, per * rate / len(Xc))))
        t0 = time.perf_counter()
        cmatvec.gamma_apply(p["kernel"], 1.0, p["ell"], Xr[:rows], Xc, Y)
        dt = time.perf_counter() - t0
        total_pairs += rows * len(Xc)
        total_time += dt
        parts.append(f"{p['method']}-{p['kernel']}: {rows} rows x {len(Xc)} cols")
    return {"value": total_pairs / total_time, "unit": "pairs/s", "cores": cmatvec.max_threads(), "kind": "oracle",
            "sample": f"FP64 C/OpenMP kernel product (oracle/cmatvec.c), b={probs[0]['block']}, " + "; ".join(parts)
            + f"; {total_pairs:.3g} pairs in {total_time:.1f} s"}


def request_pairs(d):
    """Kernel pairs of one block application for a problem descriptor."""
    p, nel = d["p"], d["nel"]
    N = int(np.prod([p + e for e in nel]))
    if d["method"] == "galerkin":
        mult = p if d["kernel"] == "exponential" else 1
        Nt = int(np.prod([p + 1 + mult * (e - 1) for e in nel]))
        return float(Nt) * Nt
    return float(N) * float(np.prod([(p + 1) * e for e in nel]))


def serve_benchmark(n_requests, rhos, cap, tol, seed=210100629):
    """Serving workload: seed-drawn K-L requests, Poisson arrivals.

    Sequential baseline: every request solved alone (ka_setup + ka_eigs +
    ka_destroy) and timed; its FIFO latencies on the arrival trace follow
    from those measured service times.  Server: the same trace through the
    continuous-batching server (ka_server_*), measured end to end."""
    import torch
    import paper_2101_00629_amd as K
    from workloads import serving_stream

    trace = serving_stream(n_requests, seed=seed, max_pairs=cap, pair_count=request_pairs)
    descs = [K.desc_from_problem({k: v for k, v in d.items() if k not in ("M", "arrival", "id", "name")},
                                 seed=1 + d["id"]) for d in trace]
    cplx = [d["method"] == "collocation" for d in trace]
    # sequential plain solves
    service, lam_seq, seq_status = [], [], []
    for i, d in enumerate(trace):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = K.Problem(descs[i])
        try:
            rc, lam, info = K.ka_eigs(prob.h, d["M"], tol=tol, maxit=60)
        except K.KAError as e:   # a failed solve is reported with its status, as the server does
            rc, lam, info = e.code, np.zeros(2 * d["M"]), {"iterations": None, "converged": 0}
        prob.close()
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        lam_seq.append(lam)
        seq_status.append((rc, info))
        if (i + 1) % 32 == 0:
            print(f"[serve] sequential {i + 1}/{n_requests} solves, {sum(service):.1f} s", file=sys.stderr, flush=True)
    service = np.array(service)
    def brief(d):
        return {k: d[k] for k in ("method", "domain", "p", "nel", "kernel", "ell", "M", "block")}
    seq_fail = [{"request": i, "status": rc, "iterations": info["iterations"], "converged": info["converged"],
                 **brief(trace[i])} for i, (rc, info) in enumerate(seq_status) if rc != 0]
    out = {"requests": n_requests, "pair_cap_per_block_product": cap, "sequential_nonzero_status": seq_fail,
           "mean_service_ms": float(service.mean() * 1e3),
           "pairs_per_block_product": {"p50": float(np.median([request_pairs(d) for d in trace])),
                                       "max": float(max(request_pairs(d) for d in trace))}}
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0, n_requests)
    for rho in rhos:
        arrivals = np.cumsum(gaps) * service.mean() / rho
        arrivals -= arrivals[0]
        # FIFO one-at-a-time on the measured service times
        done, t = np.zeros(n_requests), 0.0
        for i in range(n_requests):
            t = max(t, arrivals[i]) + service[i]
            done[i] = t
        seq_lat = done - arrivals
        # continuous-batching server
        srv = K.ka_server_create(64 << 30, 32)
        lams = []
        for i, d in enumerate(trace):
            lam = np.zeros(2 * d["M"])
            lams.append(lam)
            K.ka_server_submit(srv, descs[i], d["M"], lam, tol=tol, maxit=60, arrival_s=float(arrivals[i]), tag=i)
        print(f"[serve] server run, rho {rho:g}", file=sys.stderr, flush=True)
        import threading
        t0 = time.perf_counter()
        runner = threading.Thread(target=K.ka_server_run, args=(srv, 1200.0))
        runner.start()
        res = []
        while runner.is_alive():            # progress while the server runs (results are mutex-guarded)
            runner.join(timeout=15.0)
            res.extend(K.ka_server_poll(srv))
            print(f"[serve] rho {rho:g}: {len(res)}/{n_requests} done, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        res.extend(K.ka_server_poll(srv))
        print(f"[serve] server run done in {wall:.1f} s", file=sys.stderr, flush=True)
        res = sorted(res, key=lambda r: r["tag"])
        stats = K.ka_server_stats(srv)
        K.ka_server_destroy(srv)
        ok = [r for r in res if r["status"] == 0]
        lat = np.array([r["done_s"] - r["arrival_s"] for r in res])
        makespan = max(r["done_s"] for r in res)
        diff = 0.0
        okset = {r["tag"] for r in ok}
        for i, d in enumerate(trace):
            if i not in okset or seq_status[i][0] != 0:
                continue
            a = lams[i][0::2][:d["M"]] if cplx[i] else lams[i][:d["M"]]
            b = lam_seq[i][0::2] if cplx[i] else lam_seq[i]
            diff = max(diff, float(np.abs(a - b).max() / abs(b[0])))
        out[f"rho_{rho:g}"] = {
            "server": {"solves_per_s": n_requests / makespan, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat, 99) * 1e3), "makespan_s": makespan, "wall_s": wall,
                       "completed": len(ok), "max_active": stats["max_active"],
                       "mean_items_per_launch": stats["mean_items"]},
            "sequential": {"solves_per_s": n_requests / done[-1], "p50_ms": float(np.percentile(seq_lat, 50) * 1e3),
                           "p99_ms": float(np.percentile(seq_lat, 99) * 1e3), "makespan_s": float(done[-1])},
            "max_eig_diff_vs_alone_rel_lambda1": diff,
            "server_nonzero_status": [{"request": r["tag"], "status": r["status"],
                                       "iterations": r["info"]["iterations"], "converged": r["info"]["converged"],
                                       **brief(trace[r["tag"]])} for r in res if r["status"] != 0],
        }
    return out


def kernel_rates(warm=3, reps=10):
    """Raw fused kernel product (ka_gamma_apply) at the workload shapes, both
    precisions: median per-launch device time over `reps` launches after
    `warm` warm-up launches, HIP events on the launch stream.  Points are
    tensor grids of the workloads' point counts in the problems' order (first
    direction fastest) on the workloads' domains: the FP32 Gaussian path takes
    its centred Gram form for row blocks of small extent, so the cost depends
    on how the points are ordered.  Y is N(0,1)."""
    import torch
    import paper_2101_00629_amd as K
    from workloads import normal_block, tensor_grid_points

    shapes = [  # (name, kernel, ell, domain, row grid, column grid, b)
        ("cube p3 20^3 Galerkin Gaussian", "gaussian", 0.5, "cube", (23, 23, 23), (23, 23, 23), 16),
        ("cube p3 20^3 Galerkin exponential (C0)", "exponential", 1.0, "cube", (61, 61, 61), (61, 61, 61), 16),
        ("cube p3 20^3 collocation", "gaussian", 0.5, "cube", (23, 23, 23), (80, 80, 80), 16),
        ("annulus p4 32x32x16 Galerkin Gaussian", "gaussian", 0.5, "quarter_annulus", (36, 36, 20), (36, 36, 20), 32),
        ("annulus p4 32x32x16 Galerkin exponential (C0)", "exponential", 0.25, "quarter_annulus", (129, 129, 65),
         (129, 129, 65), 32),
        ("annulus p4 32x32x16 collocation", "gaussian", 0.5, "quarter_annulus", (36, 36, 20), (160, 160, 80), 32),
        ("cube p2 64^3 Galerkin Gaussian", "gaussian", 0.2, "cube", (66, 66, 66), (66, 66, 66), 64),
    ]
    out = []
    for name, kern, ell, dom, gr, gc, b in shapes:
        xc = torch.tensor(tensor_grid_points(gc, dom), dtype=torch.float32, device="cuda")
        xr = xc if gr == gc else torch.tensor(tensor_grid_points(gr, dom), dtype=torch.float32, device="cuda")
        nr, nc = xr.shape[0], xc.shape[0]
        y = torch.tensor(normal_block(9, nc, b, dtype=np.float32), device="cuda")
        z = torch.empty((nr, b), dtype=torch.float32, device="cuda")
        for prec, pname in ((K.KA_FP32, "fp32"), (K.KA_BF16X3, "bf16x3")):
            nbytes = K.ka_gamma_workspace(nr, nc, b, prec)
            work = torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device="cuda")
            big = nr * nc > 2e11
            nrep = 3 if big else reps
            for _ in range(1 if big else warm):
                K.ka_gamma_apply(K.KERNELS[kern], 1.0, ell, xr, xc, y, z, prec, work)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nrep)]
            for e0, e1 in ev:
                e0.record()
                K.ka_gamma_apply(K.KERNELS[kern], 1.0, ell, xr, xc, y, z, prec, work)
                e1.record()
            torch.cuda.synchronize()
            ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
            rate = nr * nc / (ms / 1e3)
            rec = {"shape": name, "rows": nr, "cols": nc, "b": b, "kernel": kern, "precision": pname,
                   "launches": nrep, "median_ms": ms, "pairs_per_s": rate,
                   "frac_valu_peak": rate / peak_pairs(kern)}
            if pname == "fp32":
                rec["frac_serial_peak"] = rate / serial_peak_pairs(kern, b)
            out.append(rec)
            print(f"[rates] {name} b={b} {pname}: {ms:.3f} ms, {rate / 1e12:.3f} Tpairs/s", file=sys.stderr,
                  flush=True)
            del work
        del xc, xr, y, z
    return out


def compare_methods(reps=3):
    """The paper's comparison (Sec. 4) on the unit cube: eigensolver time
    against the mean relative error of the 20 largest eigenvalues (eps-bar),
    for Galerkin-IBQ, collocation and standard Gauss-quadrature Galerkin.
    Example-1 analogue: L1-exponential kernel (ell = 1), p = 2, h-refinement.
    Example-2 analogue: Gaussian kernel (ell = 0.5), 6^3 elements, k-refinement
    p = 2..6.  References: the continuous spectra stored in
    tests/golden/cube_continuum_spectra.json.  Time = median over `reps` solves
    of ka_eigs (set-up excluded, as the paper times the eigensolver), FP32."""
    import torch
    import paper_2101_00629_amd as K

    with open(os.path.join(ROOT, "tests", "golden", "cube_continuum_spectra.json")) as f:
        cont = json.load(f)
    series = [("exponential", 1.0, cont["exponential_l1"]["lambda"], [(2, n) for n in (4, 6, 8, 12, 16, 24)]),
              ("gaussian", 0.5, cont["gaussian_l0.5"]["lambda"], [(p, 6) for p in (2, 3, 4, 5, 6)])]
    out = []
    for kernel, ell, ref, meshes in series:
        ref = np.array(ref)
        for p, nel in meshes:
            for method in ("galerkin", "collocation", "galerkin_gauss"):
                desc = K.make_desc(method, "cube", p, (nel, nel, nel), kernel, ell, block=16, seed=5)
                prob = K.Problem(desc)
                times = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    rc, lam, info = K.ka_eigs(prob.h, 20, tol=1e-6, maxit=80)
                    times.append(time.perf_counter() - t0)
                N, Nt, Nq, _ = K.ka_size(prob.h)
                prob.close()
                lr = lam[0::2] if method == "collocation" else lam
                eps = np.abs(lr[:20] - ref) / ref
                rec = {"kernel": kernel, "ell": ell, "p": p, "nel": nel, "method": method, "N": N,
                       "points": Nt if method == "galerkin" else Nq, "status": rc,
                       "eps_bar": float(eps.mean()), "eps_max": float(eps.max()),
                       "solve_s": float(np.median(times)), "matvecs": info["matvecs"], "pairs": info["pairs"]}
                out.append(rec)
                print(f"[compare] {kernel} p={p} nel={nel} {method}: N={N} eps_bar={rec['eps_bar']:.2e} "
                      f"t={rec['solve_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return out


def half_cylinder_benchmark(reps=2):
    """The paper's numerical examples (Sec. 4) on the thick-walled half
    cylinder (workloads.HALF_CYLINDER; one C^0 line, the middle of the half
    circle), sigma = 1, ell = 5.  Example 1: L1-exponential kernel, p = 2, the
    five meshes of Table 1 (C^0 interpolation space).  Example 2: Gaussian
    kernel, the Case 1 mesh with p = 2..6 (Table 2).  Per case and method
    (Galerkin-IBQ, collocation): N, interpolation or quadrature points, set-up
    time, eigensolver time (median of `reps` ka_eigs; the paper times the
    eigensolver), and the mean relative error eps-bar of the 20 largest
    eigenvalues against a standard Gauss-quadrature Galerkin reference on a
    finer mesh, solved on the GPU as well.  A second, coarser reference gives
    the first one's own eps-bar as a bound on how far eps-bar can be trusted."""
    import torch
    import paper_2101_00629_amd as K
    from workloads import HALF_CYLINDER, HALF_CYLINDER_EXAMPLE1, HALF_CYLINDER_EXAMPLE2, half_cylinder_net

    hc = half_cylinder_net(HALF_CYLINDER["r0"], HALF_CYLINDER["r1"], HALF_CYLINDER["length"])
    ell = HALF_CYLINDER["ell"]
    M = 20

    def solve(method, p, nel, kernel, block, n_rep, maxit=80):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = K.Problem(K.make_desc(method, "nurbs", p, nel, kernel, ell, block=block, seed=11, nurbs=hc))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        times = []
        for _ in range(n_rep):
            t0 = time.perf_counter()
            rc, lam, info = K.ka_eigs(prob.h, M, tol=1e-6, maxit=maxit)
            times.append(time.perf_counter() - t0)
        N, Nt, Nq, _ = K.ka_size(prob.h)
        prob.close()
        lr = np.asarray(lam[0::2] if method == "collocation" else lam)[:M]
        return dict(method=method, p=p, nel=list(nel), N=N, points=Nt if method == "galerkin" else Nq,
                    status=rc, setup_s=setup_s, solve_s=float(np.median(times)), matvecs=info["matvecs"],
                    pairs=info["pairs"]), lr

    examples = [("example1", "exponential", [(2, nel) for nel in HALF_CYLINDER_EXAMPLE1],
                 [(2, (126, 9, 69)), (2, (84, 6, 46))]),
                ("example2", "gaussian", HALF_CYLINDER_EXAMPLE2, [(6, (64, 2, 16)), (5, (64, 2, 16))])]
    runs, refs = [], []
    for name, kernel, cases, ref_meshes in examples:
        ref_lams = []
        for p, nel in ref_meshes:
            rec, lam = solve("galerkin_gauss", p, nel, kernel, 32, 1)
            ref_lams.append(lam)
            rec.update(example=name, kernel=kernel)
            refs.append(rec)
            print(f"[half-cylinder] {name} reference p={p} nel={nel}: N={rec['N']} points={rec['points']} "
                  f"solve {rec['solve_s']:.2f} s", file=sys.stderr, flush=True)
        ref = ref_lams[0]
        refs[-1]["eps_bar_vs_first_reference"] = float(np.mean(np.abs(ref_lams[1] - ref) / ref))
        for case, (p, nel) in enumerate(cases, 1):
            for method in ("galerkin", "collocation"):
                rec, lam = solve(method, p, nel, kernel, 16, reps)
                eps = np.abs(lam - ref) / ref
                rec.update(example=name, case=case, kernel=kernel, eps_bar=float(eps.mean()),
                           eps_first5=[float(e) for e in eps[:5]])
                runs.append(rec)
                print(f"[half-cylinder] {name} case {case} {method}: N={rec['N']} points={rec['points']} "
                      f"eps_bar={rec['eps_bar']:.2e} solve {rec['solve_s'] * 1e3:.1f} ms", file=sys.stderr,
                      flush=True)
    return dict(runs=runs, references=refs)


def measure(K, torch, name, precision, steps, warmup, tol):
    """Solve the workload's problems `warmup` + `steps` times in one precision;
    returns rates, latencies, accuracy and the kernel product's roofline."""
    probs = workload(name, precision=precision)
    handles = []
    for i, p in enumerate(probs):
        h = K.Problem(K.desc_from_problem(p, seed=1000 + i))
        handles.append(h)

    def one_step():
        out = []
        for p, h in zip(probs, handles):
            t0 = time.perf_counter()
            rc, lam, info = K.ka_eigs(h.h, p["M"], tol=tol, maxit=60)
            dt = time.perf_counter() - t0
            if rc != 0:
                raise RuntimeError(f"ka_eigs returned {rc} for {p['name']}: {info}")
            out.append((lam, info, dt))
        return out

    for _ in range(warmup):
        one_step()
    for h in handles:
        K.ka_profile_reset(h.h)
        K.ka_profile_enable(h.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(steps):
        results.append(one_step())
        print(f"[bench] {name} {precision} step {k + 1}/{steps}: {time.perf_counter() - t0:.2f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = [K.ka_profile_read(h.h) for h in handles]
    for h in handles:
        K.ka_profile_enable(h.h, False)

    pairs = sum(info["pairs"] for step in results for (_, info, _) in step)
    lat = np.array([dt for step in results for (_, _, dt) in step]) * 1e3
    nsolves = len(lat)
    # eigenvalue accuracy of the last step against the stored FP64 reference spectra
    eig = {}
    worst = 0.0
    for p, (lam, info, _) in zip(probs, results[-1]):
        ref = reference_spectrum(name, p)
        lr = lam[0::2] if p["method"] == "collocation" else lam
        e = floored_rel_errors(ref, lr)
        worst = max(worst, float(e.max()))
        eig[f"{p['method']}-{p['kernel']}"] = {"max_floored_rel_err": float(e.max()),
                                               "max_raw_rel_err": float(floored_rel_errors(ref, lr, 0.0).max()),
                                               "matvecs": info["matvecs"], "cycles": info["iterations"],
                                               "floor_accepted": info["floor_accepted"]}
    # roofline of the fused kernel product: pairs of every timed launch over
    # their summed device time (HIP events on the launch stream)
    gl_pairs = sum(pp for (_, _, pp) in prof)
    gl_ms = sum(ms for (_, ms, _) in prof)
    launches = sum(n for (n, _, _) in prof)
    achieved = gl_pairs / (gl_ms / 1e3)

    def harmonic(rate):   # pairs-weighted harmonic mean of per-problem peaks
        return gl_pairs / sum(pp / rate(p) for p, (_, _, pp) in zip(probs, prof))

    out = {"probs": probs, "pairs": pairs, "elapsed": elapsed, "lat": lat, "nsolves": nsolves, "eig": eig,
           "worst": worst, "achieved": achieved, "launches": launches, "gl_ms": gl_ms,
           "valu_peak": harmonic(lambda p: peak_pairs(p["kernel"])),
           "mfma_peak": harmonic(lambda p: mfma_pairs(p["block"])),
           "serial_peak": harmonic(lambda p: serial_peak_pairs(p["kernel"], p["block"])),
           "flops_per_pair": gl_pairs and sum(2.0 * p["block"] * pp for p, (_, _, pp) in zip(probs, prof)) / gl_pairs}
    for h in handles:
        h.close()
    return out


def roofline(res, name, precision):
    """Roofline record of the fused kernel product.  FP32: the contraction's
    2 b flops per pair on the FP32 matrix cores (157.3 TFLOP/s) and the tile
    evaluation's VALU slots do not overlap on gfx950; whichever takes longer
    per pair is the bound ("mfma" for b = 64).  BF16x3: against the dense
    BF16 matrix peak (2.5 PFLOP/s) with the three products' 6 b flops per
    pair; with the Gram form its VALU work per pair is the exp and the hi/lo
    split, and the matrix cores are the busiest unit (about 0.5 of the cycles
    at b = 64, VALU issue about 0.4)."""
    a = res["achieved"]
    rec = {"kernel": "gamma_f32_kernel" if precision == "fp32" else "gamma_bf16x3_kernel",
           "launches": res["launches"], "kernel_ms": res["gl_ms"],
           "kernel_share_of_step": res["gl_ms"] / 1e3 / res["elapsed"],
           "pairs_per_s": a, "valu_peak_pairs_per_s": res["valu_peak"], "valu_frac": a / res["valu_peak"]}
    if precision == "fp32":
        rec.update(mfma_frac=a / res["mfma_peak"], serial_valu_mfma_peak_pairs_per_s=res["serial_peak"],
                   serial_frac=a / res["serial_peak"])
        if res["mfma_peak"] < res["valu_peak"]:
            flops = a * res["flops_per_pair"]
            rec.update(bound="mfma", achieved=flops / 1e12, peak=MFMA_F32_FLOPS / 1e12, unit="TFLOP/s",
                       frac=flops / MFMA_F32_FLOPS)
        else:
            rec.update(bound="alu", achieved=a, peak=res["valu_peak"], unit="pairs/s", frac=a / res["valu_peak"])
        rec.update(traffic=measured_traffic(name), traffic_unit="HBM bytes per launch",
                   algorithmic_bytes_per_launch=TRAFFIC[name]["algorithmic_bytes"])
    else:
        flops = a * 3.0 * res["flops_per_pair"]
        rec.update(bound="mfma", achieved=flops / 1e12, peak=MFMA_BF16_FLOPS / 1e12, unit="TFLOP/s",
                   frac=flops / MFMA_BF16_FLOPS)
    return rec


def nurbs_benchmark(reps=2):
    """General NURBS volumes at workload size: the quarter annulus given as a
    control net against the closed-form annulus (p = 4, 32 x 32 x 16, the
    annulus workload's mesh), and a curved volume with per-point weights
    (p = 3, 20^3 elements).  Per problem: set-up time (ka_setup, host geometry
    evaluation included), median solve time of ka_eigs, the kernel product's
    rate and roofline fraction (HIP events), and for the annulus the largest
    floored eigenvalue difference between the two descriptions."""
    import torch
    import paper_2101_00629_amd as K
    from workloads import nurbs_annulus_net, nurbs_blob_net

    blob = nurbs_blob_net(11, n=(6, 6, 6), degree=(3, 3, 3), wiggle=0.04)
    cases = []
    for method, M, b in (("collocation", 100, 32), ("galerkin", 100, 32)):
        base = dict(method=method, p=4, nel=(32, 32, 16), kernel="gaussian", ell=0.5, block=b)
        cases.append((f"annulus p4 32x32x16 {method}, closed form", base | dict(domain="quarter_annulus"), M, "ann"))
        cases.append((f"annulus p4 32x32x16 {method}, NURBS control net", base | dict(domain="nurbs", nurbs=nurbs_annulus_net()),
                      M, "ann"))
    for method in ("collocation", "galerkin"):
        cases.append((f"curved volume (per-point weights) p3 20^3 {method}",
                      dict(method=method, domain="nurbs", nurbs=blob, p=3, nel=(20, 20, 20), kernel="gaussian",
                           ell=0.5, block=16), 50, None))
    out, ann = [], {}
    for name, kw, M, group in cases:
        cplx = kw["method"] == "collocation"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = K.Problem(K.make_desc(seed=3, **kw))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        times = []
        for r in range(reps + 1):
            if r == 1:
                K.ka_profile_reset(prob.h)
                K.ka_profile_enable(prob.h, True)
            t0 = time.perf_counter()
            rc, lam, info = K.ka_eigs(prob.h, M, tol=1e-5, maxit=80)
            if r >= 1:
                times.append(time.perf_counter() - t0)
        n_l, ms, pairs = K.ka_profile_read(prob.h)
        prob.close()
        lr = lam[0::2] if cplx else lam
        rec = {"problem": name, "status": rc, "M": M, "block": kw["block"], "setup_s": setup_s,
               "solve_s": float(np.median(times)), "matvecs": info["matvecs"],
               "kernel_pairs_per_s": pairs / (ms / 1e3), "kernel_frac_valu": pairs / (ms / 1e3) / peak_pairs("gaussian")}
        if group:
            key = kw["method"]
            if key in ann:
                rec["max_floored_diff_vs_closed_form"] = float(floored_rel_errors(ann[key], lr).max())
            else:
                ann[key] = lr
        out.append(rec)
        print(f"[nurbs] {name}: setup {setup_s:.2f} s, solve {rec['solve_s'] * 1e3:.1f} ms, "
              f"kernel {rec['kernel_pairs_per_s'] / 1e12:.2f} Tpairs/s", file=sys.stderr, flush=True)
    return out


def kl_sample_benchmark(reps=3):
    """K-L field sampling at workload size: eigenpairs by ka_eigs on the
    device, then ka_kl_sample of S fields on a parametric tensor grid
    (N(0,1) draws from a seeded generator, passed in).  Reported per case:
    median wall time of the whole call (norms, eigenfunction values, field
    product; it synchronizes), fields/s, and the rates the field product
    alone would need at that time (2 P S M flops; P S 8 bytes written)."""
    import torch
    import paper_2101_00629_amd as K
    from workloads import annulus_p4, cube_p3_20

    cases = []
    p = annulus_p4("galerkin", "gaussian")
    cases.append(("annulus p4 32x32x16 Galerkin Gaussian, M=100", p, p["M"], (64, 64, 32), 1000))
    p = cube_p3_20("galerkin", "exponential")
    cases.append(("cube p3 20^3 Galerkin exponential (C0), M=50", p, p["M"], (64, 64, 64), 1000))
    p = cube_p3_20("collocation", "gaussian")
    cases.append(("cube p3 20^3 collocation Gaussian, M=50", p, p["M"], (64, 64, 64), 1000))
    out = []
    for name, prob_d, M, npts, S in cases:
        cplx = prob_d["method"] == "collocation"
        prob = K.Problem(K.desc_from_problem(prob_d, seed=17))
        V = torch.zeros((M, prob.N), dtype=torch.float64, device="cuda")
        rc, lam, info = K.ka_eigs(prob.h, M, tol=1e-5, maxit=80, V=V)
        lam = lam[0::2] if cplx else lam
        grid = [np.linspace(0.0, 1.0, n) for n in npts]
        P = int(np.prod(npts))
        gen = torch.Generator(device="cuda")
        gen.manual_seed(23)
        xi = torch.randn((S, M), dtype=torch.float64, device="cuda", generator=gen)
        F = torch.empty((S, P), dtype=torch.float64, device="cuda")
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            K.ka_kl_sample(prob.h, np.maximum(lam, 0.0), V, grid, xi, F, mu=0.0)
            if r:
                times.append(time.perf_counter() - t0)
        prob.close()
        t = float(np.median(times))
        rec = {"case": name, "eigs_status": rc, "M": M, "grid": list(npts), "points": P, "samples": S,
               "call_ms": t * 1e3, "fields_per_s": S / t, "product_tflops_at_call_time": 2.0 * P * S * M / t / 1e12,
               "output_gb_per_s_at_call_time": P * S * 8 / t / 1e9}
        out.append(rec)
        print(f"[kl] {name}: {P} points x {S} samples, {t * 1e3:.1f} ms per call", file=sys.stderr, flush=True)
        del V, xi, F
    return out


def latency(lat):
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "max": float(lat.max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--workload", default="cube64", choices=sorted(WORKLOADS),
                    help="cube64: the 64^3 cube (default); cube20: the four 20^3 cube problems")
    ap.add_argument("--no-serve-leg", action="store_true", help="skip the short serving leg of the default line")
    ap.add_argument("--serve-requests", type=int, default=128, help="requests of the serving leg")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split-bf16", action="store_true",
                    help="skip the second pass of the workload in split-BF16 precision")
    ap.add_argument("--serve", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rho", default="0.5,1.5")
    ap.add_argument("--pair-cap", type=float, default=1e11)
    ap.add_argument("--compare", action="store_true",
                    help="the paper's method comparison (time vs eigenvalue error) on the cube instead")
    ap.add_argument("--kernel-rates", action="store_true",
                    help="time the raw kernel product at every workload shape instead")
    ap.add_argument("--kl-sample", action="store_true",
                    help="K-L field sampling at workload size (ka_kl_sample) instead")
    ap.add_argument("--nurbs", action="store_true",
                    help="general NURBS volumes at workload size (annulus as a control net, curved volume) instead")
    ap.add_argument("--half-cylinder", action="store_true",
                    help="the paper's Examples 1 and 2 on the half cylinder (time vs eps-bar) instead")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus 1): multi-GPU execution is not implemented; the path would shard "
              "the kernel product by rows, one all-gather of Z per block product", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2101_00629_amd as K

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.compare:
        print(json.dumps({"metric": "eigensolver time vs mean relative error of 20 eigenvalues", "n_gpus": 1,
                          "data": "synthetic (unit cube)", "dtype": "f32", "runs": compare_methods()}), flush=True)
        return
    if args.kernel_rates:
        print(json.dumps({"metric": "fused kernel product pairs/s at the workload shapes", "n_gpus": 1,
                          "data": "synthetic (tensor-grid points in the problems' order, N(0,1) blocks)", "unit": "pairs/s",
                          "rates": kernel_rates()}), flush=True)
        return
    if args.kl_sample:
        print(json.dumps({"metric": "K-L field samples on a parametric grid", "n_gpus": 1, "data": "synthetic",
                          "dtype": "f64", "runs": kl_sample_benchmark()}), flush=True)
        return
    if args.nurbs:
        print(json.dumps({"metric": "K-L solves on general NURBS volumes", "n_gpus": 1, "data": "synthetic",
                          "dtype": "f32", "runs": nurbs_benchmark()}), flush=True)
        return
    if args.half_cylinder:
        print(json.dumps({"metric": "half-cylinder examples: eigensolver time vs eps-bar of 20 eigenvalues",
                          "n_gpus": 1, "data": "synthetic (half cylinder, Sec. 4 meshes)", "dtype": "f32",
                          **half_cylinder_benchmark()}), flush=True)
        return
    if args.serve:
        res = serve_benchmark(args.requests, [float(r) for r in args.rho.split(",")], args.pair_cap, args.tol)
        print(json.dumps({"metric": "K-L solves/s + p99 latency (serving)", "n_gpus": 1, "data": "synthetic",
                          "dtype": "f32", **res}), flush=True)
        return
    name = args.workload
    res = measure(K, torch, name, args.precision, args.steps, args.warmup, args.tol)
    probs = res["probs"]
    line = {
        "metric": METRIC,
        "value": res["pairs"] / res["elapsed"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[name], "solves_per_step": len(probs), "tol": args.tol,
                   "precision": args.precision},
        "solves_per_s": res["nsolves"] / res["elapsed"],
        "latency_ms": latency(res["lat"]),
        "eig_err": {"max_floored_rel_err": res["worst"], "bar": 1e-6 if args.precision == "fp32" else 1e-5,
                    "per_problem": res["eig"]},
        "roofline": roofline(res, name, args.precision),
    }
    if args.precision == "fp32" and not args.no_split_bf16:
        # the same workload with the contraction in split hi/lo BF16 (its bar: 1e-5)
        nb = max(1, min(args.steps, 3))
        rb = measure(K, torch, name, "bf16x3", nb, 1, args.tol)
        line["split_bf16"] = {
            "value": rb["pairs"] / rb["elapsed"], "unit": "pairs/s", "steps": nb,
            "solves_per_s": rb["nsolves"] / rb["elapsed"], "latency_ms": latency(rb["lat"]),
            "eig_err": {"max_floored_rel_err": rb["worst"], "bar": 1e-5,
                        "per_problem": {k: v["max_floored_rel_err"] for k, v in rb["eig"].items()}},
            "roofline": roofline(rb, name, "bf16x3")}
    if not args.no_serve_leg:
        sv = serve_benchmark(args.serve_requests, [1.5], args.pair_cap, args.tol)
        r = sv["rho_1.5"]
        line["serving"] = {
            "requests": sv["requests"], "rho": 1.5, "pair_cap_per_block_product": args.pair_cap,
            "server": {k: r["server"][k] for k in ("solves_per_s", "p50_ms", "p99_ms", "completed", "max_active")},
            "sequential": {k: r["sequential"][k] for k in ("solves_per_s", "p50_ms", "p99_ms")},
            "max_eig_diff_vs_alone_rel_lambda1": r["max_eig_diff_vs_alone_rel_lambda1"],
            "nonzero_status": len(r["server_nonzero_status"]) + len(sv["sequential_nonzero_status"])}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(probs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
