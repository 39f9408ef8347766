"""Benchmark of the solver's hot path on one MI355X.

One step = one full solve of Algorithm 1 on the dense 50000 x 4000 workload (coherent:
20% of rows scaled by 1e3, b ~ N(0,1); hashing s = 3 after the randomised Hadamard
transform, gamma = 1.7 so m = 6800; Householder QR of the sketch; LSQR on A R^-1 to the
(TC-lsqr) tolerance 1e-10): ski_sketch + ski_factor + ski_solve with A and b already in
HBM.  Prints one JSON line on stdout (everything else goes to stderr).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-mixed]
                       [--no-sparse] [--no-very-sparse] [--no-rankdef] [--no-batched]
                       [--no-seeds] [--rankdef-only] [--batched-only] [--very-sparse-only]
                       [--sweep]
                       [--sketch-study] [--cache-ceiling]
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time & sketch GB/s at 50000x4000; mixed vs FP64 at equal 1e-10 residual"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lsqr_pass_dense_50000x4000_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2105_11815_amd", "csrc", "lsqr.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_dense():
    import workloads
    c = workloads.CASES["dense"]
    A, b = workloads.dense_coherent(n=c["n"], d=c["d"], case=c["case"])
    return A, b, c


def one_solve(P, S, At, bt, **kw):
    S.sketch(At, bt, **kw).factor()
    X, infos, rc = S.solve()
    return X, infos[0], rc


def cpu_model():
    """The host CPU's model name as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_phases(A, b, cfg, iters, threads, cols=(60, 180), reps=3, its=4):
    """Per-phase seconds of one oracle solve on the dense workload, with the BLAS pool
    limited to `threads` (None: all of them).  Measured on the real A and b:
      sketch -- the oracle's Walsh-Hadamard + hashing of the first c columns of [A b]
                for the two column counts in `cols` (median of `reps` runs each); the
                transform and the hashing act column by column, so the time is a fixed
                part (drawing S_h and D) plus a per-column part, and the line through
                the two points gives the full d+1 columns;
      qr     -- the oracle's Householder QR (LAPACK) of an m x (d+1) matrix, once (its
                cost does not depend on the values: no pivoting);
      lsqr   -- `its` iterations of the oracle's preconditioned LSQR on the full A, median
                seconds per iteration over `reps` runs, times `iters` iterations."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import lls, sketch as sk
    n, d, m, s = A.shape[0], A.shape[1], cfg["m"], cfg["s"]
    with threadpool_limits(limits=threads):
        used = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        tc = []
        for c in cols:
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                sk.sketch_dense(A[:, : c - 1], b, m, s, seed=2002)
                ts.append(time.perf_counter() - t0)
            tc.append(float(np.median(ts)))
        # fixed part (S_h and D: the same for any column count) plus a per-column part
        per_col = (tc[1] - tc[0]) / (cols[1] - cols[0])
        t_sketch = tc[0] + per_col * (d + 1 - cols[0])
        SA = np.random.default_rng(0).standard_normal((m, d + 1))
        t0 = time.perf_counter()
        R, _, _ = lls.factor(SA, d)
        t_qr = time.perf_counter() - t0
        tl = []
        for _ in range(reps):
            t0 = time.perf_counter()
            lls.lsqr_precond(A, R, b.copy(), 0.0, its)
            tl.append((time.perf_counter() - t0) / its)
        t_iter = float(np.median(tl))
    total = t_sketch + t_qr + t_iter * iters
    return {"threads": int(used), "s_per_solve": round(total, 3),
            "sketch_s": round(t_sketch, 3), "sketch_sample_s": [round(t, 3) for t in tc],
            "qr_s": round(t_qr, 3),
            "lsqr_s": round(t_iter * iters, 3), "lsqr_s_per_iter": round(t_iter, 4)}


def cpu_baseline(A, b, cfg, iters):
    """The oracle as it stands, timed phase by phase on the host (cpu_phases), once with
    one BLAS thread (the sequential mode of the paper's experiments) and once with all of
    the host's threads; `value` is the all-threads rate."""
    seq = cpu_phases(A, b, cfg, iters, threads=1)
    par = cpu_phases(A, b, cfg, iters, threads=None)
    return {
        "value": 1.0 / par["s_per_solve"],
        "unit": "solves/s",
        "cores": par["threads"],
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "all_threads": par,
        "sequential": dict(seq, value=1.0 / seq["s_per_solve"]),
        "sample": (f"measured per phase on the real A and b: oracle sketch of 60 and of 180 "
                   f"of the {A.shape[1] + 1} columns (median of 3 each; fixed + per-column "
                   f"line to all columns), "
                   f"one QR of a {cfg['m']}x{A.shape[1] + 1} matrix, 4 LSQR iterations on "
                   f"the full A (median of 3, x{iters} iterations, the oracle's and the "
                   f"GPU's count on this workload)"),
    }


def pass_kernel_sha256():
    """SHA-256 of the fused pass kernel's source text (its block of lsqr.hip), so that the
    counter record stays valid across edits elsewhere in the file."""
    text = open(KERNEL_SRC, encoding="utf-8").read()
    a = text.index("// fused dense pass:")
    b = text.index("// g[c] = sum_g gpart[g][c]", a)
    return hashlib.sha256(text[a:b].encode("utf-8")).hexdigest()


def traffic_for_pass(n_launch_bytes):
    """HBM bytes per launch of the fused pass from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on the reference copy), or None
    when absent or taken on a different version of the kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                rec[key.strip()] = val.strip()
        if rec.get("kernel_source_sha256") != pass_kernel_sha256():
            return None
        return int(float(rec["bytes_per_launch"]))
    except Exception:
        return None


def sparse_run(P, torch):
    """The sparse 200000 x 5000 workload (CSR, power-law rows): a warm-up solve, the median
    of three timed solves, the optimality certificate recomputed in FP64 on the host, and a
    per-class breakdown from one more (profiled) solve."""
    import scipy.sparse as sp
    import workloads
    c = workloads.CASES["sparse"]
    n, d = c["n"], c["d"]
    rp, ci, va, b = workloads.sparse_power_law(n=n, d=d, case=c["case"])
    dev = lambda a, t: torch.as_tensor(a).to(device="cuda", dtype=t)
    Acsr = ("csr", dev(rp, torch.int64), dev(ci, torch.int32), dev(va, torch.float64), (n, d))
    bt = dev(b, torch.float64)
    kw = dict(m=c["m"], s=c["s"], seed=2003, tau_r=1e-10, hadamard=False)
    S = P.Solver()
    one_solve(P, S, Acsr, bt, **kw)
    torch.cuda.synchronize()
    times, infos = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        X, info, rc = one_solve(P, S, Acsr, bt, **kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        infos.append(info)
    S.set_profiling(True)
    one_solve(P, S, Acsr, bt, **kw)
    torch.cuda.synchronize()
    prof = S.profile()
    S.set_profiling(False)
    S.close()
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    x = X[:, 0].cpu().numpy()
    r = b - A @ x
    cert = float(np.linalg.norm(A.T @ r) / (sp.linalg.norm(A) * np.linalg.norm(r)))
    info = infos[-1]
    return {"workload": f"sparse {n}x{d} CSR, nnz {int(rp[-1])}, power-law rows (mean 10, max 500) "
                        f"+ 1e-6 identity rows, b = 1; 2-hashing, m {c['m']}; Householder QR; "
                        "LSQR with CSR products to 1e-10",
            "ms_median": round(float(np.median(times)), 3), "ms_all": [round(t, 3) for t in times],
            "iters": int(info["iters"]), "status": rc, "optimality": cert,
            "ms_sketch": round(float(info["ms_sketch"]), 3),
            "ms_factor": round(float(info["ms_factor"]), 3),
            "ms_solve": round(float(info["ms_solve"]), 3),
            "kernel_ms": {k: {"ms_total": round(v[0], 3), "launches": v[1]}
                          for k, v in prof.items() if v[1]}}


def very_sparse_run(P, torch):
    """The very sparse 40000 x 8000 workload (2 entries per column, 2-hashing, m 11200):
    the sparse QR of the sketch (SKI_QR_SPARSE) against the dense QR of the same sketch;
    a warm-up and the median of three timed solves for each, the optimality certificate
    recomputed in FP64 on the host, the factor's shape and a per-class breakdown of one
    more (profiled) sparse solve."""
    import scipy.sparse as sp
    import workloads
    c = workloads.CASES["very_sparse"]
    n, d = c["n"], c["d"]
    rp, ci, va, b = workloads.very_sparse(n, d, c["per_col"], case=c["case"])
    dev = lambda a, t: torch.as_tensor(a).to(device="cuda", dtype=t)
    Acsr = ("csr", dev(rp, torch.int64), dev(ci, torch.int32), dev(va, torch.float64), (n, d))
    bt = dev(b, torch.float64)
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    anorm = sp.linalg.norm(A)
    out = {"workload": f"very sparse {n}x{d} CSR, {c['per_col']} entries per column (row j and "
                       f"uniform rows), N(0,1), b ~ N(0,1); 2-hashing, m {c['m']}; LSQR with CSR "
                       "products to 1e-10"}
    for form in ("sparse", "auto"):
        kw = dict(m=c["m"], s=c["s"], seed=2009, tau_r=1e-10, hadamard=False, qr_panel=form)
        S = P.Solver()
        one_solve(P, S, Acsr, bt, **kw)
        torch.cuda.synchronize()
        times, infos = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            X, info, rc = one_solve(P, S, Acsr, bt, **kw)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
        x = X[:, 0].cpu().numpy()
        r = b - A @ x
        res = {"ms_median": round(float(np.median(times)), 3),
               "ms_all": [round(t, 3) for t in times], "iters": int(infos[-1]["iters"]),
               "status": rc,
               "optimality": float(np.linalg.norm(A.T @ r) / (anorm * np.linalg.norm(r))),
               "ms_sketch": round(float(infos[-1]["ms_sketch"]), 3),
               "ms_factor": round(float(infos[-1]["ms_factor"]), 3),
               "ms_solve": round(float(infos[-1]["ms_solve"]), 3)}
        if form == "sparse":
            st = S.factor_stats()
            res.update(leaf_fronts=st["leaf_fronts"], root=st["root"])
            S.set_profiling(True)
            one_solve(P, S, Acsr, bt, **kw)
            torch.cuda.synchronize()
            prof = S.profile()
            S.set_profiling(False)
            res["kernel_ms"] = {k: {"ms_total": round(v[0], 3), "launches": v[1]}
                                for k, v in prof.items() if v[1]}
        S.close()
        out["sparse_qr" if form == "sparse" else "dense_qr"] = res
    out["speedup_sparse_over_dense"] = round(out["dense_qr"]["ms_median"] /
                                             out["sparse_qr"]["ms_median"], 3)
    # larger sketches: only the sparse form takes m above 12288 (its root front stays
    # within the dense QR's limit); a tighter embedding means fewer LSQR steps
    out["sparse_qr_gamma"] = {}
    for gamma in (2.0, 3.0):
        m = int(math.ceil(gamma * d - 1e-9))
        kw = dict(m=m, s=c["s"], seed=2009, tau_r=1e-10, hadamard=False, qr_panel="sparse")
        S = P.Solver()
        one_solve(P, S, Acsr, bt, **kw)
        torch.cuda.synchronize()
        times, infos = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            X, info, rc = one_solve(P, S, Acsr, bt, **kw)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
        st = S.factor_stats()
        S.close()
        x = X[:, 0].cpu().numpy()
        r = b - A @ x
        out["sparse_qr_gamma"][str(gamma)] = {
            "m": m, "ms_median": round(float(np.median(times)), 3), "iters": int(infos[-1]["iters"]),
            "status": rc, "optimality": float(np.linalg.norm(A.T @ r) / (anorm * np.linalg.norm(r))),
            "ms_factor": round(float(infos[-1]["ms_factor"]), 3),
            "ms_solve": round(float(infos[-1]["ms_solve"]), 3),
            "leaf_fronts": st["leaf_fronts"], "root": st["root"]}
    return out


def rankdef_run(P, torch):
    """The rank-deficient 50000 x 4000 workload (rank 3500) through the column-pivoted
    factorisation: a warm-up solve, the median of three timed solves, the rank found,
    the optimality certificate recomputed in FP64, and a per-class breakdown from one more
    (profiled) solve."""
    import workloads
    c = workloads.CASES["rankdef"]
    A, b, _ = workloads.rank_deficient(n=c["n"], d=c["d"], rank=c["rank"], case=c["case"])
    At = torch.as_tensor(A).to("cuda")
    bt = torch.as_tensor(b).to("cuda")
    del A
    kw = dict(gamma=c["gamma"], m=c["m"], s=c["s"], seed=2006, tau_r=1e-10, hadamard=True,
              qr_panel="pivoted")
    S = P.Solver()
    one_solve(P, S, At, bt, **kw)
    torch.cuda.synchronize()
    times, infos = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        X, info, rc = one_solve(P, S, At, bt, **kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        infos.append(info)
    perm, p = S.get_pivots()
    S.set_profiling(True)
    one_solve(P, S, At, bt, **kw)
    torch.cuda.synchronize()
    prof = S.profile()
    S.set_profiling(False)
    S.close()
    x = X[:, 0]
    r = bt - At @ x
    cert = float((At.T @ r).norm() / (At.norm() * r.norm()))
    zero_outside = bool((x[torch.as_tensor(perm[p:], device="cuda")] == 0).all().item())
    info = infos[-1]
    # the minimal-norm form (complete orthogonal decomposition): same workload, median of 3
    kwc = dict(kw, qr_panel="cod")
    S = P.Solver()
    one_solve(P, S, At, bt, **kwc)
    torch.cuda.synchronize()
    tc, ic = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        Xc, infc, rcc = one_solve(P, S, At, bt, **kwc)
        torch.cuda.synchronize()
        tc.append((time.perf_counter() - t0) * 1e3)
        ic.append(infc)
    S.close()
    xc = Xc[:, 0]
    rc_ = bt - At @ xc
    cod = {"ms_median": round(float(np.median(tc)), 3), "ms_all": [round(t, 3) for t in tc],
           "iters": int(ic[-1]["iters"]), "status": rcc,
           "optimality": float((At.T @ rc_).norm() / (At.norm() * rc_.norm())),
           "norm_x": float(xc.norm()), "norm_x_basic": float(x.norm()),
           "ms_sketch": round(float(ic[-1]["ms_sketch"]), 3),
           "ms_factor": round(float(ic[-1]["ms_factor"]), 3),
           "ms_solve": round(float(ic[-1]["ms_solve"]), 3)}
    del At, bt
    torch.cuda.empty_cache()
    return {"workload": f"dense {c['n']}x{c['d']} of rank {c['rank']} (zero, copied and "
                        "combined columns, shuffled), 20% rows x1e3, b~N(0,1); Hadamard + "
                        f"3-hashing, m {c['m']}; column-pivoted QR truncated at rcond 1e-12; "
                        "LSQR on A_J R11^-1 to 1e-10",
            "ms_median": round(float(np.median(times)), 3), "ms_all": [round(t, 3) for t in times],
            "rank": int(p), "iters": int(info["iters"]), "status": rc, "optimality": cert,
            "x_zero_outside_J": zero_outside,
            "ms_sketch": round(float(info["ms_sketch"]), 3),
            "ms_factor": round(float(info["ms_factor"]), 3),
            "ms_solve": round(float(info["ms_solve"]), 3),
            "kernel_ms": {k: {"ms_total": round(v[0], 3), "launches": v[1]}
                          for k, v in prof.items() if v[1]},
            "minimal_norm_cod": cod}


def sweep_run(P, torch):
    """Sketch size and hashing density on the GPU (gamma = m/d and s): for the dense
    50000 x 4000 and the sparse 200000 x 5000 workloads, one warm-up and one timed solve per
    (gamma, s), with the time of each step, the LSQR iterations and the optimality
    certificate recomputed in FP64.  m stays within the 12288 rows the library supports."""
    import scipy.sparse as sp
    import workloads
    out = {}

    def run(label, A_arg, bt, certf, d, gammas, ss, base):
        rows = []
        for s in ss:
            for g in gammas:
                m = int(math.ceil(g * d - 1e-9))
                if m > 12288:
                    continue
                kw = dict(base, m=m, s=s)
                S = P.Solver()
                try:
                    one_solve(P, S, A_arg, bt, **kw)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    X, info, rc = one_solve(P, S, A_arg, bt, **kw)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3
                finally:
                    S.close()
                rows.append(dict(gamma=g, s=s, m=m, ms=round(ms, 3), iters=int(info["iters"]),
                                 status=int(rc), ms_sketch=round(info["ms_sketch"], 3),
                                 ms_factor=round(info["ms_factor"], 3),
                                 ms_solve=round(info["ms_solve"], 3),
                                 optimality=certf(X[:, 0])))
                log(f"{label} " + json.dumps(rows[-1]))
        return rows

    A, b, cfg = workload_dense()
    At = torch.as_tensor(A).to("cuda")
    bt = torch.as_tensor(b).to("cuda")
    del A

    def cert_dense(x):
        r = bt - At @ x
        return float((At.T @ r).norm() / (At.norm() * r.norm()))

    out["dense_50000x4000"] = run("dense", At, bt, cert_dense, cfg["d"],
                                  [1.3, 1.5, 1.7, 2.0, 2.5, 3.0], [1, 2, 3],
                                  dict(seed=2002, tau_r=1e-10, hadamard=True))
    del At, bt
    torch.cuda.empty_cache()
    c = workloads.CASES["sparse"]
    n, d = c["n"], c["d"]
    rp, ci, va, b = workloads.sparse_power_law(n=n, d=d, case=c["case"])
    dev = lambda a, t: torch.as_tensor(a).to(device="cuda", dtype=t)
    Acsr = ("csr", dev(rp, torch.int64), dev(ci, torch.int32), dev(va, torch.float64), (n, d))
    bt = dev(b, torch.float64)
    Ah = sp.csr_matrix((va, ci, rp), shape=(n, d))
    anorm = sp.linalg.norm(Ah)

    def cert_sparse(x):
        xh = x.cpu().numpy()
        r = b - Ah @ xh
        return float(np.linalg.norm(Ah.T @ r) / (anorm * np.linalg.norm(r)))

    out["sparse_200000x5000"] = run("sparse", Acsr, bt, cert_sparse, d,
                                    [1.2, 1.4, 1.5, 1.7, 2.0, 2.4], [1, 2, 3],
                                    dict(seed=2003, tau_r=1e-10, hadamard=False))
    return out


def sketch_study(P, torch):
    """Preconditioner quality kappa(A R^-1) from the GPU's sketch and QR (R copied back;
    kappa by a host SVD of A R^-1) on the paper's 4000 x 400 test types: hashing against
    row sampling after the transform on the coherent dense type, and s = 1, 2, 3 (s-hashing
    and its variant) on the incoherent and semi-coherent sparse types (CSR input, no
    transform)."""
    import scipy.linalg as sla
    import scipy.sparse as sp
    import workloads

    def kappa(A, R):
        sv = np.linalg.svd(sla.solve_triangular(R, A.T, trans="T").T, compute_uv=False)
        return float(sv[0] / sv[-1])

    def run(A, b, m, s, kind, dense, transform=True):
        n, d = A.shape
        S = P.Solver()
        try:
            if dense:
                S.sketch(torch.as_tensor(A).to("cuda"), torch.as_tensor(b).to("cuda"), m=m, s=s,
                         seed=31, hadamard=transform, hash_kind=kind)
            else:
                C = sp.csr_matrix(A)
                dv = lambda a, t: torch.as_tensor(a).to(device="cuda", dtype=t)
                S.sketch(("csr", dv(C.indptr.astype(np.int64), torch.int64),
                          dv(C.indices.astype(np.int32), torch.int32), dv(C.data, torch.float64),
                          (n, d)), dv(b, torch.float64), m=m, s=s, seed=31, hadamard=False,
                         hash_kind=kind)
            S.factor()
            R = S.get_R()[0]
        except P.SkiError as e:
            return None if "rank" in str(e).lower() or "ERANK" in str(e) else str(e)
        finally:
            S.close()
        return kappa(A, R)

    out = {}
    A, b = workloads.coherent_dense(4000, 400)
    rows = []
    for ratio in (1.25, 1.5, 2, 3, 4, 6, 8):
        m = int(ratio * 400)
        rows.append(dict(m_over_d=ratio, hashing_s1=run(A, b, m, 1, "hash", True),
                         sampling=run(A, b, m, 1, "sample", True),
                         hashing_s1_dht=run(A, b, m, 1, "hash", True, "dht"),
                         sampling_dht=run(A, b, m, 1, "sample", True, "dht")))
        log("coherent dense " + json.dumps(rows[-1]))
    out["coherent_dense_4000x400"] = rows
    for name, A in (("inco_sparse_4000x400", workloads.inco_sparse(4000, 400)),
                    ("semico_sparse_4000x400", workloads.semico_sparse(4000, 400)[0])):
        b = np.ones(4000)
        rows = []
        for ratio in (1.25, 1.5, 2, 3, 4):
            m = int(ratio * 400)
            r = dict(m_over_d=ratio)
            for s in (1, 2, 3):
                r[f"hash_s{s}"] = run(A, b, m, s, "hash", False)
                if s > 1:
                    r[f"variant_s{s}"] = run(A, b, m, s, "variant", False)
            rows.append(r)
            log(f"{name} " + json.dumps(r))
        out[name] = rows
    # the two transforms on the dense 50000 x 4000 workload: sketch and whole solve
    Ad, bd, cfg = workload_dense()
    At = torch.as_tensor(Ad).to("cuda")
    bt = torch.as_tensor(bd).to("cuda")
    del Ad
    tr = {}
    for name, hv in (("walsh_hadamard", True), ("hartley", "dht")):
        kw = dict(m=cfg["m"], s=cfg["s"], seed=2002, tau_r=1e-10, hadamard=hv)
        S = P.Solver()
        one_solve(P, S, At, bt, **kw)
        torch.cuda.synchronize()
        ts, infos = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            X, info, rc = one_solve(P, S, At, bt, **kw)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
        S.close()
        x = X[:, 0]
        r = bt - At @ x
        tr[name] = dict(ms=round(float(np.median(ts)), 3),
                        ms_sketch=round(float(np.median([i["ms_sketch"] for i in infos])), 3),
                        iters=int(infos[-1]["iters"]),
                        optimality=float((At.T @ r).norm() / (At.norm() * r.norm())))
        log(f"dense 50000x4000 {name} " + json.dumps(tr[name]))
    out["transforms_dense_50000x4000"] = tr
    return out


def batched_run(P, torch):
    """The batched workload (20000 x 1000, 32 right-hand sides, FP64): the forward solve
    through the multi-right-hand-side LSQR (its A products are MFMA GEMMs), then the
    backward: the adjoint solve Z = (A^T A)^-1 G by CG with the forward's R and the two
    gradients.  Median of three after a warm-up; the forward's A products are timed by
    the profiler classes and priced at 2 n d k flops each."""
    import workloads
    c = workloads.CASES["batched"]
    A, B, G = workloads.batched(n=c["n"], d=c["d"], k=c["k"], case=c["case"])
    At, Bt, Gt = (torch.as_tensor(v).to("cuda") for v in (A, B, G))
    kw = dict(m=c["m"], s=c["s"], seed=2005, tau_r=1e-10, hadamard=True)
    n, d, k = A.shape[0], A.shape[1], B.shape[1]
    fw, bw, its, cg_its = [], [], 0, 0
    for rep in range(4):
        S = P.Solver()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.sketch(At, Bt, **kw).factor()
        X, infos, rc = S.solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Z, zinfos, zrc = S.solve_normal(Gt)
        gA, gB = S.gradients(X, Bt, Z)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        S.close()
        if rep:
            fw.append((t1 - t0) * 1e3)
            bw.append((t2 - t1) * 1e3)
        its = max(i["iters"] for i in infos)
        cg_its = max(i["iters"] for i in zinfos)
    R = Bt - At @ X
    cert = float(((At.T @ R).norm(dim=0) / (At.norm() * R.norm(dim=0))).max())
    # per iteration two GEMMs of 2 n d k flops each (A Z and A^T U)
    tf = 4.0 * n * d * k * its / (float(np.median(fw)) * 1e-3) / 1e12
    return {"workload": f"dense {n}x{d}, {k} right-hand sides B ~ N(0,1), loss weight G ~ N(0,1); "
                        f"Hadamard + {c['s']}-hashing, m {c['m']}; LSQR to 1e-10 on all columns; "
                        "adjoint CG with the same R, then grad_A and grad_B",
            "forward_ms": round(float(np.median(fw)), 3), "backward_ms": round(float(np.median(bw)), 3),
            "forward_ms_all": [round(t, 3) for t in fw], "backward_ms_all": [round(t, 3) for t in bw],
            "lsqr_iters_max": int(its), "cg_iters_max": int(cg_its), "optimality_worst": cert,
            "forward_lsqr_gemm_TFLOPs_lower_bound": round(tf, 2)}


def cache_ceiling(torch):
    """Read+write rate of a device-to-device copy whose source and destination together
    take `mb` MB, for footprints from well inside the 256 MB last-level cache to well
    beyond it (median of 20 timed copies after 5 untimed): the rate the sketch's slab
    passes can reach while their slab stays cache-resident, against the HBM rate."""
    out = {}
    for mb in (16, 32, 64, 128, 192, 256, 512, 2048):
        nel = mb * (1 << 20) // 16  # two buffers of mb/2 MB each
        a = torch.empty(nel, dtype=torch.float64, device="cuda").normal_()
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        ts = []
        for _ in range(20):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        out[f"{mb}MB"] = {"ms": round(ms, 5), "GBps_read_plus_write": round(2 * nel * 8 / (ms * 1e-3) / 1e9, 1)}
        del a, b
        torch.cuda.empty_cache()
    return out


def mixed_runs(P, torch, At, bt, base_kw, forms, label):
    """Time one solve per precision form (after a warm-up solve) and recompute the
    residual and the optimality certificate ||A^T r|| / (||A||_F ||r||) in FP64."""
    out, xs = {}, {}
    for name, kw in forms:
        S = P.Solver()
        try:
            one_solve(P, S, At, bt, **base_kw, **kw)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, info, rc = one_solve(P, S, At, bt, **base_kw, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
        finally:
            S.close()
        x = X[:, 0]
        r = bt - At @ x
        cert = float((At.T @ r).norm() / (At.norm() * r.norm()))
        xs[name] = x
        out[name] = dict(ms=round(ms, 3), iters=int(info["iters"]), status=int(rc),
                         rnorm=float(r.norm()), optimality=cert,
                         ms_sketch=round(info["ms_sketch"], 3),
                         ms_factor=round(info["ms_factor"], 3),
                         ms_solve=round(info["ms_solve"], 3))
    if "fp64" in xs:
        for name in xs:
            if name != "fp64":
                out[name]["x_rel_diff_vs_fp64"] = float((xs[name] - xs["fp64"]).norm()
                                                        / xs["fp64"].norm())
    log(f"{label}: " + json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-very-sparse", action="store_true")
    ap.add_argument("--very-sparse-only", action="store_true")
    ap.add_argument("--no-rankdef", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-seeds", action="store_true")
    ap.add_argument("--rankdef-only", action="store_true",
                    help="only the rank-deficient workload (for profiling); prints its record")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched 32-right-hand-side workload (for profiling)")
    ap.add_argument("--sweep", action="store_true",
                    help="only the gamma/s sweep of the dense and sparse workloads; prints it")
    ap.add_argument("--cache-ceiling", action="store_true",
                    help="only the copy rate against the copy's footprint (cache vs HBM)")
    ap.add_argument("--sketch-study", action="store_true",
                    help="only the preconditioner-quality study of the sketch variants")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path, so --gpus "
              "must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_11815_amd as P

    if args.rankdef_only:
        print(json.dumps({"rankdef_50000x4000": rankdef_run(P, torch)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_20000x1000_k32": batched_run(P, torch)}), flush=True)
        return
    if args.very_sparse_only:
        print(json.dumps({"very_sparse_40000x8000": very_sparse_run(P, torch)}), flush=True)
        return
    if args.sweep:
        print(json.dumps({"gamma_s_sweep": sweep_run(P, torch)}), flush=True)
        return
    if args.cache_ceiling:
        print(json.dumps({"cache_ceiling": cache_ceiling(torch)}), flush=True)
        return
    if args.sketch_study:
        print(json.dumps({"sketch_study": sketch_study(P, torch)}), flush=True)
        return

    log("generating the dense 50000x4000 workload ...")
    A, b, cfg = workload_dense()
    At = torch.as_tensor(A).to("cuda")
    bt = torch.as_tensor(b).to("cuda")
    torch.cuda.synchronize()
    kw = dict(gamma=cfg["gamma"], m=cfg["m"], s=cfg["s"], seed=2002, tau_r=1e-10,
              hadamard=True)
    n, d, k = A.shape[0], A.shape[1], 1

    # reference device-to-device copy of A (read and write 8nd bytes): the achievable
    # streaming rate, and the calibration point for the HBM byte counters
    ref = torch.empty_like(At)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ref.copy_(At)
    ev0.record()
    ref.copy_(At)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * At.numel() * 8 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del ref

    S = P.Solver()
    for _ in range(args.warmup):
        one_solve(P, S, At, bt, **kw)
    torch.cuda.synchronize()
    # only the dominant kernel is bracketed by events, in the last two timed steps (its
    # average launch time feeds the roofline): an event pair costs ~11 us of device time
    # per iteration, so the other steps and launches run without event records
    prof_steps = min(2, args.steps)
    iters_sum = iters_prof = 0
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        if step == args.steps - prof_steps:
            S.set_profiling(True, classes=["lsqr_pass"])
        X, info, rc = one_solve(P, S, At, bt, **kw)
        iters_sum += int(info["iters"])
        if step >= args.steps - prof_steps:
            iters_prof += int(info["iters"])
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = S.profile()
    # per-class breakdown from one more solve, outside the timed region
    S.set_profiling(True)
    one_solve(P, S, At, bt, **kw)
    torch.cuda.synchronize()
    prof_all = S.profile()
    S.set_profiling(False)
    S.close()
    ms_step = wall * 1e3 / args.steps
    info = infos[-1]
    log(f"ms/step {ms_step:.3f}  iters {info['iters']}  status {rc}  profile {prof}")

    # correctness of the timed solve (recomputed in FP64)
    x = X[:, 0]
    r = bt - At @ x
    cert = float((At.T @ r).norm() / (At.norm() * r.norm()))

    # sketch bandwidth: A and b read once, SA written once
    m = cfg["m"]
    sk_bytes = 8 * n * (d + k) + 8 * m * (d + k)
    sk_ms = float(np.median([i["ms_sketch"] for i in infos]))
    sketch_gbps = sk_bytes / (sk_ms * 1e-3) / 1e9

    # roofline of the dominant kernel: the fused LSQR pass (A once, u read and written)
    pass_ms, pass_cnt = prof["lsqr_pass"]
    pass_bytes = 8 * n * d + 16 * n
    pass_avg_ms = pass_ms / max(iters_prof, 1)
    achieved = pass_bytes / (pass_avg_ms * 1e-3) / 1e9
    traffic = traffic_for_pass(pass_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": traffic, "kernel": "k_lsqr_pass<16, 2> (fused u = A z - c u, g = A^T u)",
                "bytes_per_launch": pass_bytes, "avg_launch_ms": round(pass_avg_ms, 5),
                "launches_timed": pass_cnt, "lsqr_iterations_timed": iters_prof,
                "timed_steps_with_events": prof_steps}
    # per kernel class, one solve (profiled apart from the timed steps)
    phases = {kname: {"ms_total": round(v[0], 3), "launches": v[1]}
              for kname, v in prof_all.items() if v[1]}

    out = {
        "metric": METRIC, "value": round(1e3 / ms_step, 4), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dense 50000x4000, 20% rows x1e3, b~N(0,1); Hadamard + "
                               "3-hashing, gamma 1.7 (m=6800); Householder QR; LSQR to 1e-10",
                   "n": n, "d": d, "m": m, "s": cfg["s"], "tau_r": 1e-10},
        "time_to_solution_ms": round(ms_step, 3),
        "sketch_GBps": round(sketch_gbps, 1), "sketch_ms": round(sk_ms, 3),
        "factor_ms": round(float(np.median([i["ms_factor"] for i in infos])), 3),
        "solve_ms": round(float(np.median([i["ms_solve"] for i in infos])), 3),
        "lsqr_iters": int(info["iters"]), "optimality_certificate": cert,
        "rnorm": float(r.norm()), "kernel_ms": phases, "roofline": roofline,
        "copy_GBps_reference": round(copy_gbps, 1),
    }

    # three sketch seeds on the same A: the spread of the time to solution
    seeds = {}
    S = P.Solver()
    for sd in (() if args.no_seeds else (2002, 3002, 4002)):
        kws = dict(kw, seed=sd)
        one_solve(P, S, At, bt, **kws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            Xs, infs, _ = one_solve(P, S, At, bt, **kws)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        seeds[str(sd)] = dict(ms_median=round(float(np.median(ts)), 3),
                              ms_min=round(min(ts), 3), ms_max=round(max(ts), 3),
                              iters=int(infs["iters"]))
    S.close()
    if seeds:
        out["seeds"] = seeds

    if not args.no_batched:
        log("batched 20000x1000 workload ...")
        out["batched_20000x1000_k32"] = batched_run(P, torch)
        torch.cuda.empty_cache()

    if not args.no_sparse:
        log("sparse 200000x5000 workload ...")
        out["sparse_200000x5000"] = sparse_run(P, torch)
        torch.cuda.empty_cache()

    if not args.no_very_sparse:
        log("very sparse 40000x8000 workload (sparse and dense QR of the sketch) ...")
        out["very_sparse_40000x8000"] = very_sparse_run(P, torch)
        torch.cuda.empty_cache()

    if not args.no_rankdef:
        log("rank-deficient 50000x4000 workload ...")
        out["rankdef_50000x4000"] = rankdef_run(P, torch)

    if not args.no_mixed:
        forms = [("fp64", {}), ("fp32", dict(sketch_prec="fp32", qr_prec="fp32")),
                 ("bf16", dict(sketch_prec="bf16", qr_prec="bf16", it_max=3000)),
                 ("fp64sketch_fp32qr", dict(sketch_prec="fp64", qr_prec="fp32", it_max=3000))]
        out["mixed_dense_50000x4000"] = mixed_runs(P, torch, At, bt, kw, forms, "dense")
        del At, bt
        torch.cuda.empty_cache()
        import workloads
        c4 = workloads.CASES["illcond"]
        log("generating the ill-conditioned 50000x7000 workload on the GPU ...")
        A4, b4 = workloads.illcond(n=c4["n"], d=c4["d"], case=c4["case"], device="cuda")
        torch.cuda.synchronize()
        kw4 = dict(gamma=c4["gamma"], m=c4["m"], s=c4["s"], seed=2004, tau_r=1e-10,
                   hadamard=True)
        out["mixed_illcond_50000x7000"] = mixed_runs(P, torch, A4, b4, kw4, forms, "illcond")
        del A4, b4
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(A, b, cfg, int(info["iters"]))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
