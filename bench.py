"""Benchmark: solves/s of the non-nested multilevel smoothed Schwarz FGMRES
solve on one MI355X, with the dominant kernel's roofline and the CPU oracle
timed beside it.

One step = one full solve of the three-level jittered 48^3 / 24^3 / 10^3
problem (log-Gaussian kappa, 64 subdomains, FP64) to relative residual
1e-8, starting from x0 = 0, with the factors resident in HBM.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {8: 78.6, 4: 157.3}  # dense FP64 / FP32 matrix peaks
PMC_SUMMARY = os.path.join(ROOT, "profiles", "{kernel}_cube48_{prec}_pmc.md")


def source_hash():
    """Hash of the smoother kernel's sources (the kernel, the device headers
    it includes, and the host functions that lay out its subdomains and its
    work items): counter summaries taken from an older kernel are not
    reported."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_08981_amd", "csrc")
    for name in ("ras.hip", "devcommon.h", "devtypes.h"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    for name, sig in (("api.hip", b"static std::vector<int32_t> ras_tasks("),
                      ("api.hip", b"static std::vector<int32_t> xpanel_tasks("), ("host_setup.cpp", b"void build_blocks(")):
        text = open(os.path.join(csrc, name), "rb").read()
        i = text.find(sig)
        h.update(text[i:text.find(b"\n}\n", i)] if i >= 0 else b"")
    return h.hexdigest()[:16]


def load_traffic(prec, kernel="k_ras"):
    """HBM bytes per launch of the fine-level smoother from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a plain copy of known size), or None when absent or stale."""
    path = PMC_SUMMARY.format(kernel=kernel, prec=prec)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip().lstrip("- ").strip()] = v.strip()
    if kv.get("ras_hip_sha256_16") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def xpanel_bytes(h, level, s_bytes):
    """Algorithmic bytes of one inverse-panel smoother application on
    `level`: X_p = J_p^{-1} E_o read once in its stored symmetric form, the
    overlap rows (n_v n_o values) and the lower triangle of the owned block
    (n_o (n_o + 1) / 2), plus the gathered input, the index map and the
    scattered owned output."""
    owner, sets = h.partition(level)
    owner = np.asarray(owner)
    n = np.array([len(S) for S in sets], dtype=np.float64)
    no = np.array([np.count_nonzero(owner[np.asarray(S)] == p) for p, S in enumerate(sets)], dtype=np.float64)
    if level == h.L - 1:
        no = n
    vals = (n - no) * no + no * (no + 1) / 2
    return float(np.sum(vals) * s_bytes + np.sum(n) * (s_bytes + 4) + np.sum(no) * s_bytes)


def ras_bytes(h, level, s_bytes):
    """Algorithmic bytes of one smoother application on `level`: the forward
    sweep reads L on and below the diagonal (n_p (n_p + 1) / 2 values), the
    backward sweep U on and above it in the owned rows only (n_o (n_o + 1) / 2:
    the restriction keeps x_o = inv(U_oo) y_o, and the owned rows come last),
    plus the gathered input, the index map and the scattered owned output.
    The coarsest level (one subdomain, every row owned) reads n^2 + n."""
    owner, sets = h.partition(level)
    owner = np.asarray(owner)
    n = np.array([len(S) for S in sets], dtype=np.float64)
    no = np.array([np.count_nonzero(owner[np.asarray(S)] == p) for p, S in enumerate(sets)], dtype=np.float64)
    vals = n * (n + 1) / 2 + no * (no + 1) / 2
    return float(np.sum(vals) * s_bytes + np.sum(n) * (s_bytes + 4) + np.sum(no) * s_bytes)


def ilu_bytes(h, level, s_bytes):
    """Algorithmic bytes of one ILU smoother application on `level`: every
    factor entry once (value and local column), the row starts, diagonal
    positions, level orders and index map of every row, the gathered input
    and the scattered owned output."""
    li = h.level_info(level)
    return float(li.ilu_nnz * (s_bytes + 4) + li.s_total * (4 * 5 + s_bytes) + li.ninterior * li.ncomp * s_bytes)


def lu_flops(h, level):
    """Algorithmic flops of the level's dense subdomain LUs: (2/3) n_p^3 each
    (unpadded sizes; the kernels also run the 64-padding), plus, with inverse
    panels, their block substitutions: the forward one over the owned
    columns' unit vectors (n_o^3 / 3) and the backward one of every owned
    column (n_p^2 n_o); on the coarsest level, whose whole inverse is kept
    as its lower triangle, n^3 / 3 + n^3 / 2."""
    from paper_2412_08981_amd import nnms

    owner, sets = h.partition(level)
    owner = np.asarray(owner)
    n = np.array([len(S) for S in sets], dtype=np.float64)
    fl = float(np.sum(2.0 / 3.0 * n ** 3))
    if h.level_info(level).dense_apply == nnms.INVERSE:
        if level == h.L - 1:
            fl += float(np.sum(n ** 3 / 3.0 + n ** 3 / 2.0))
        else:
            no = np.array([np.count_nonzero(owner[np.asarray(S)] == p) for p, S in enumerate(sets)],
                          dtype=np.float64)
            fl += float(np.sum(no ** 3 / 3.0 + n * n * no))
    return fl


def spmv_bytes(h, level, s_bytes):
    li = h.level_info(level)
    return float(li.nnz * (4 + s_bytes) + 4 * (li.ndof + 1) + 3 * li.ndof * s_bytes)


def prolong_bytes(h, level, s_bytes):
    """z_f += P z_c: four (index, weight) pairs per fine row (barycentric) or
    one per entry of P (MLS), the coarse vector once, the fine vector read
    and written."""
    from paper_2412_08981_amd import nnms

    li, lc = h.level_info(level), h.level_info(level + 1)
    nf, nc = li.ndof, lc.ndof
    if li.transfer == nnms.MLS:
        return float(li.p_nnz * (4 + s_bytes) + nc * s_bytes + 2 * nf * s_bytes)
    return float(nf * (16 + 4 * s_bytes) + nc * s_bytes + 2 * nf * s_bytes)


def restrict_bytes(h, level, s_bytes):
    """r_c = P^T t: the CSR of P^T over coarse rows, t once, r_c written."""
    li, lc = h.level_info(level), h.level_info(level + 1)
    return float(li.r_nnz * (4 + s_bytes) + 4 * (lc.ndof + 1) + (li.ndof + lc.ndof) * s_bytes)


def cpu_baseline(pb, seconds_cap=60.0, mls_alpha=None, elasticity=False, mls_clip=False):
    """The FP64 oracle (NumPy/SciPy, LAPACK) on the host cores: setup once,
    then one full solve of the same problem; solves/s = 1 / solve time."""
    import workloads as W
    from oracle import problem as oprob
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    if elasticity:
        from oracle import elasticity as oel
        oh = oel.build(pb, nu=W.ELASTIC_NU, f=W.ELASTIC_FORCE)
    else:
        oh = oprob.build(pb, mls_alpha=mls_alpha, mls_clip=mls_clip)
    t1 = time.perf_counter()
    res = oprob.solve(oh)
    t2 = time.perf_counter()
    return {
        "value": 1.0 / (t2 - t1),
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"one full solve ({res.iterations} FGMRES iterations) of the same problem ({pb.name}) after "
                  f"the oracle's setup ({t1 - t0:.1f} s, not counted)",
    }, oh, res


def cpu_baseline_extra():
    """The oracle on the other workloads, bounded samples: the two-level 16^3
    problem (setup, then the solve timed over 5 repeats) and one instance of
    each of the two smallest fine sizes of the batched instances (24^3 and
    32^3; the batch's larger instances take minutes each on the host)."""
    import workloads as W
    from oracle import problem as oprob

    out = {}
    pb = W.cube16_two_level()
    oh = oprob.build(pb)
    t = time.perf_counter()
    for _ in range(5):
        res = oprob.solve(oh)
    out["cube16_two_level"] = {"solves_per_s": round(5 / (time.perf_counter() - t), 3), "iterations": res.iterations,
                               "sample": "5 solves of the two-level 16^3/6^3 problem (kappa = 1, 8 subdomains)"}
    probs = W.batched_instances(count=32)
    picked, seen = [], set()
    for i, p in enumerate(probs):
        n = int(p.meshes[0].n)
        if n in (24, 32) and n not in seen:
            seen.add(n)
            picked.append((i, p))
    el, its = 0.0, []
    for i, p in picked:
        oh = oprob.build(p)
        t = time.perf_counter()
        res = oprob.solve(oh)
        el += time.perf_counter() - t
        its.append(res.iterations)
    out["batched_instances_sample"] = {
        "solves_per_s": round(len(picked) / el, 3), "iterations": its,
        "sample": f"instances {[i for i, _ in picked]} of the 32 batched instances (fine n = "
                  f"{[int(p.meshes[0].n) for _, p in picked]}), solved one after the other in FP64 (the oracle has no "
                  "FP32 path); the full batch mixes in 40^3 to 64^3 instances, so its oracle rate is lower"}
    return out


def hierarchy_options(args, nnms):
    """Transfer and subdomain-solver keywords of nnms.Hierarchy from the
    command line, and a short description for the workload name."""
    kw = {"transfer": nnms.MLS if args.transfer == "mls" else nnms.BARYCENTRIC, "mls_alpha": args.mls_alpha,
          "subsolver": nnms.ILU if args.subsolver == "ilu" else nnms.LU,
          "ilu_fill": [int(k) for k in args.ilu_fill.split(",")],
          "dense_apply": nnms.INVERSE if args.dense_apply == "inverse" else nnms.SWEEPS}
    desc = ""
    if args.transfer == "mls":
        desc += f", MLS transfer (scale {args.mls_alpha} x mean coarse edge)"
    if args.subsolver == "ilu":
        desc += f", ILU({args.ilu_fill}) subdomain solves"
    if args.dense_apply == "inverse":
        desc += ", dense subdomain solves through inverse panels"
    return kw, desc


def smoother_bytes(h, level, s_bytes):
    """Algorithmic bytes of one smoother application, dense LU or ILU."""
    from paper_2412_08981_amd import nnms

    li = h.level_info(level)
    if li.subsolver == nnms.ILU and level < h.L - 1:
        return ilu_bytes(h, level, s_bytes)
    if li.dense_apply == nnms.INVERSE:
        return xpanel_bytes(h, level, s_bytes)
    return ras_bytes(h, level, s_bytes)


def batched_leg(args, steps):
    """The batched instances (config of the batched workload) solved `steps`
    times as one batch and once one after the other: (batched solves/s,
    sequential solves/s, iterations, max relres, every batched result
    bitwise equal to its solve alone, tuning, ms per batched solve)."""
    import torch
    import workloads as W
    from paper_2412_08981_amd import nnms

    probs = W.batched_instances(count=args.batch)
    hkw, hdesc = hierarchy_options(args, nnms)
    t0 = time.perf_counter()
    hs, ss, bs = [], [], []
    for pb in probs:
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its, precision=nnms.MIXED, **hkw)
        s = nnms.System(h, pb.kappa, 1.0)
        hs.append(h)
        ss.append(s)
        bs.append(s.rhs())
    from paper_2412_08981_amd import autotune
    tuning = autotune.tune(ss[0], cache=args.tuning_cache)
    torch.cuda.synchronize()
    log(f"[bench batched] {len(ss)} instances set up in {time.perf_counter() - t0:.1f} s, "
        f"sizes {[int(pb.meshes[0].n) for pb in probs]}")
    xs, infos = nnms.solve_batch(ss, bs)  # warm-up (captures the graph)
    t = time.perf_counter()
    for _ in range(steps):
        xs, infos = nnms.solve_batch(ss, bs)
    el = (time.perf_counter() - t) / steps
    t = time.perf_counter()
    alone = [s.solve(b) for s, b in zip(ss, bs)]
    el_seq = time.perf_counter() - t
    same = all(np.array_equal(x, a[0]) for x, a in zip(xs, alone))
    its = [i.iterations for i in infos]
    res = {"solves_per_s": len(ss) / el, "sequential_solves_per_s": len(ss) / el_seq, "iterations": its,
           "max_relres": max(i.relres for i in infos), "bitwise_equal_alone": bool(same), "tuning": tuning,
           "ms_per_batch": 1e3 * el, "count": len(ss), "desc": hdesc}
    for s in ss:
        s.destroy()
    return res


def run_batched(args):
    """Batched parametric instances of uneven mesh and subdomain sizes (fine
    n in {24,32,40,48,64}, three non-nested levels each), mixed precision,
    solved together in one launch sequence per Arnoldi step (HIP graph) vs
    one after the other."""
    r = batched_leg(args, args.steps)
    out = {
        "metric": "solves/s to rel-res 1e-8 (batched)",
        "value": round(r["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": round(r["ms_per_batch"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{r['count']} parametric instances, fine n in {{24,32,40,48,64}}, 3 non-nested "
                               "levels, mixed precision, one batched launch sequence per Arnoldi step (HIP graph)"
                               + r["desc"],
                   "sequential_solves_per_s": round(r["sequential_solves_per_s"], 3),
                   "batch_gain": round(r["solves_per_s"] / r["sequential_solves_per_s"], 3),
                   "iterations": r["iterations"], "max_relres": r["max_relres"],
                   "batch_equals_alone_bitwise": r["bitwise_equal_alone"], "tuning": r["tuning"]},
    }
    print(json.dumps(out))


def run_serving(args):
    """Serving: Poisson arrivals of parametric solve requests over three
    resident hierarchies (jittered 32^3, 64^3, 96^3 fine meshes, three levels
    each), device-memory budget admission, continuous batching.  The closed-
    loop capacity is measured first (requests all queued at t = 0), then an
    open-loop Poisson trace at 0.7x that capacity gives p50 / p99 latency.
    Both precisions are run on the same requests."""
    import torch
    import workloads as W
    from paper_2412_08981_amd import nnms
    from paper_2412_08981_amd.serve import Request, Server

    sizes = (32, 64, 96)
    centres = W.serving_centres()
    t, hs_choice, mus = W.serving_trace(nreq=args.requests, rate=1.0, sizes=sizes)
    res = {}
    hkw, hdesc = hierarchy_options(args, nnms)
    for precision in ("mixed", "fp64"):
        prec = nnms.MIXED if precision == "mixed" else nnms.FP64
        t0 = time.perf_counter()
        hier, keep = {}, []
        for n in sizes:
            meshes = W.served_hierarchy(n)
            ms = [nnms.Mesh.from_workload(m) for m in meshes]
            nps = [W.nparts_rule(m.nv) for m in meshes[:-1]]
            # PyTorch's caching allocator: releasing a finished request's
            # system or a batch plan does not synchronise the device
            hier[n] = nnms.Hierarchy(ms, nps, precision=prec, torch_alloc=True, **hkw)
            keep.append(ms)
        from paper_2412_08981_amd import autotune
        sb = 8 if prec == nnms.FP64 else 4
        kern = {}
        for n in sizes:
            sample = nnms.System(hier[n], W.KappaField("loggauss", centres=centres, mu=mus[0], width=W.KAPPA_WIDTH))
            autotune.tune(sample, cache=args.tuning_cache)
            # fine-level kernels of each resident hierarchy (the 96^3 residual
            # moves ~160 MB: bandwidth-bound, unlike the 21 MB one of 48^3)
            h = hier[n]
            msr = sample.time_kernel(1, 0, reps=20)
            mss = sample.time_kernel(0, 0, reps=5)
            msp = sample.time_kernel(2, 0, reps=20)
            msq = sample.time_kernel(3, 0, reps=20)
            kern[f"{n}^3"] = {"residual_l0_ms": round(msr, 4),
                              "residual_l0_GBs": round(spmv_bytes(h, 0, sb) / (msr * 1e-3) / 1e9, 1),
                              "prolong_l0_ms": round(msp, 4),
                              "prolong_l0_GBs": round(prolong_bytes(h, 0, sb) / (msp * 1e-3) / 1e9, 1),
                              "restrict_l0_ms": round(msq, 4),
                              "restrict_l0_GBs": round(restrict_bytes(h, 0, sb) / (msq * 1e-3) / 1e9, 1),
                              "smoother_l0_ms": round(mss, 4),
                              "smoother_l0_GBs": round(smoother_bytes(h, 0, sb) / (mss * 1e-3) / 1e9, 1)}
            sample.destroy()
        log(f"[bench serving] {precision}: kernels {kern}")
        log(f"[bench serving] {precision}: hierarchies set up in {time.perf_counter() - t0:.1f} s; bytes per request "
            f"{ {n: round(h.system_bytes() / 2**30, 2) for n, h in hier.items()} } GiB")

        def make(ids, times):
            return [Request(int(i), int(hs_choice[i]),
                            W.KappaField("loggauss", centres=centres, mu=mus[i], width=W.KAPPA_WIDTH), float(tt))
                    for i, tt in zip(ids, times)]

        # closed-loop capacity: a burst of requests at t = 0
        nb = min(args.requests, args.burst)
        srv = Server(hier, args.budget_gib * 2**30)
        st_cap = srv.run(make(range(nb), np.zeros(nb)))
        cap = st_cap["solves_per_s"]
        # open loop: Poisson arrivals at 0.7x capacity (exponential gaps, seeded)
        gaps = np.random.default_rng(5001).exponential(1.0 / (0.7 * cap), size=args.requests)
        srv = Server(hier, args.budget_gib * 2**30)
        st = srv.run(make(range(args.requests), np.cumsum(gaps)))
        st["rate_per_s"] = 0.7 * cap
        st["capacity_solves_per_s"] = cap
        st["batch_forms"] = srv.batch_forms
        st["steps"] = srv.steps
        st["kernels"] = kern
        st["capacity_run"] = {k: st_cap[k] for k in ("host_s_batch_forms", "host_s_steps", "host_s_results",
                                                     "numeric_setup_ms_mean", "p50_ms")}
        res[precision] = st
        log(f"[bench serving] {precision}: {st}")
        del srv, hier, keep
        torch.cuda.synchronize()
    m = res["mixed"]
    out = {
        "metric": "solves/s to rel-res 1e-8 (continuous-batching serving), p50/p99 latency",
        "value": round(m["capacity_solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": round(1e3 / m["capacity_solves_per_s"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} Poisson requests over resident jittered 32^3/64^3/96^3 "
                               f"hierarchies (3 levels), budget {args.budget_gib} GiB, mixed precision" + hdesc,
                   "p50_ms": m.get("p50_ms"), "p99_ms": m.get("p99_ms"), "open_loop_solves_per_s": m.get("solves_per_s"),
                   "fp64": res["fp64"],
                   "mixed": m,
                   "mixed_over_fp64_capacity": round(m["capacity_solves_per_s"] / res["fp64"]["capacity_solves_per_s"], 3)},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--workload", default="cube48", choices=["cube48", "cube16", "batched", "serving", "served96"],
                    help="cube48: the three-level 48^3 problem (default); cube16: the two-level 16^3/6^3 problem "
                         "(kappa = 1, 8 subdomains); batched: ragged parametric instances; serving: continuous "
                         "batching of Poisson arrivals; served96: the largest served hierarchy (96^3/48^3/20^3, "
                         "512 + 64 subdomains) as one system")
    ap.add_argument("--requests", type=int, default=60, help="requests of the serving trace")
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2412_08981_amd", "tuning.json"),
                    help="launch-shape cache (measured on first use)")
    ap.add_argument("--burst", type=int, default=18, help="requests of the closed-loop capacity run")
    ap.add_argument("--budget-gib", type=float, default=160.0, help="device-memory budget of the serving loop")
    ap.add_argument("--batch", type=int, default=32, help="instances of the batched workload")
    ap.add_argument("--transfer", default="barycentric", choices=["barycentric", "mls"],
                    help="transfer between levels: barycentric P1 interpolation or moving least squares")
    ap.add_argument("--mls-alpha", type=float, default=1.0, help="MLS initial scale / mean coarse edge length")
    ap.add_argument("--mls-clip", action="store_true",
                    help="with the MLS transfer: clip every neighbourhood to the overlapping subdomain of the "
                         "target's processor (Section 3.2)")
    ap.add_argument("--coarsen", default="", metavar="M[,M2]",
                    help="derive the coarse levels from the fine mesh by Algorithm 1 with M rounds per level "
                         "(a list gives the rounds of each coarse level)")
    ap.add_argument("--subsolver", default="lu", choices=["lu", "ilu"],
                    help="subdomain solver of the smoother: dense LU or ILU(k)")
    ap.add_argument("--ilu-fill", default="2,0", help="ILU level of fill per smoothed level (finest first)")
    ap.add_argument("--dense-apply", default=None, choices=["sweeps", "inverse"],
                    help="dense-LU subdomain solves applied by forward/backward sweeps over the factors, or "
                         "through the stored owned columns of each subdomain inverse (inverse panels; about "
                         "twice the numeric setup).  Default: inverse, except for the serving workload, whose "
                         "requests are each assembled once and solved once (sweeps)")
    ap.add_argument("--physics", default="poisson", choices=["poisson", "elasticity"],
                    help="default workload: the scalar 48^3 problem, or P1 linear elasticity (three unknowns per "
                         "vertex, field-split transfers) on 32^3/16^3/7^3 meshes")
    ap.add_argument("--nparts", default="", metavar="P0[,P1]",
                    help="default workload: subdomains per smoothed level (e.g. 64,64: the same count on every "
                         "smoothed level, as the paper partitions every level)")
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the mixed-precision and batched legs")
    ap.add_argument("--factor-only", action="store_true",
                    help="time the fine level's numeric factorisation a few times (for counter runs)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run the copy reference and the fine-level smoother a few times each (for counter runs)")
    ap.add_argument("--transfers-only", action="store_true",
                    help="time the prolongation and restriction of every level at the tuned shapes (JSON line)")
    args = ap.parse_args()
    if args.dense_apply is None:
        args.dense_apply = "sweeps" if args.workload == "serving" else "inverse"
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2412_08981_amd import nnms

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    torch.cuda.init()
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "serving":
        return run_serving(args)
    elastic = args.physics == "elasticity"
    if elastic:
        pb = W.cube32_elasticity(args.precision)
    elif args.workload == "cube16":
        pb = W.cube16_two_level()
        pb.precision = args.precision
    elif args.workload == "served96":
        # the largest served hierarchy as a single system (96^3 / 48^3 / 20^3)
        ms96 = W.served_hierarchy(96)
        pb = W.Problem("served96", ms96, [W.nparts_rule(m.nv) for m in ms96[:-1]], W.kappa_draw(5003, 5004),
                       precision=args.precision)
    else:
        pb = W.cube48_three_level(args.precision)
    prec = nnms.MIXED if args.precision == "mixed" else nnms.FP64
    t0 = time.perf_counter()
    meshes = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    fine_mesh = pb.meshes[0]
    coarsened = None
    rounds = [int(r) for r in args.coarsen.split(",")] if args.coarsen else []
    if rounds:
        rounds += [rounds[-1]] * (len(pb.meshes) - 1 - len(rounds))
        # coarse levels from the fine mesh (Algorithm 1), not meshed on their own
        meshes = meshes[:1]
        for l in range(1, len(pb.meshes)):
            c, _ = meshes[-1].coarsen(rounds[l - 1], l)
            meshes.append(c)
        coarsened = []
        for l, m in enumerate(meshes):
            xyz_l, tets_l, d_l = m.read()
            coarsened.append(W.Mesh(xyz_l, tets_l, d_l, 0))
        pb = W.Problem(pb.name + "-coarsened", coarsened, [W.nparts_rule(m.nv) if l else pb.nparts[0]
                                                          for l, m in enumerate(coarsened[:-1])],
                       pb.kappa, precision=pb.precision)
        log(f"[bench] coarsened levels (Algorithm 1, rounds {rounds}): vertices "
            f"{[m.nv for m in coarsened]}, interior {[int((m.dirichlet == 0).sum()) for m in coarsened]}")
    if args.nparts:
        nps = [int(p) for p in args.nparts.split(",")]
        pb = W.Problem(pb.name, pb.meshes, nps + pb.nparts[len(nps):], pb.kappa, precision=pb.precision)
    mls_mode = args.transfer == "mls"
    ilu_mode = args.subsolver == "ilu"
    xinv_mode = args.dense_apply == "inverse"
    ilu_fill = [int(k) for k in args.ilu_fill.split(",")]
    h = nnms.Hierarchy(meshes, pb.nparts, overlap=pb.overlap, its=pb.its, precision=prec,
                       transfer=nnms.MLS if mls_mode else nnms.BARYCENTRIC, mls_alpha=args.mls_alpha,
                       subsolver=nnms.ILU if ilu_mode else nnms.LU, ilu_fill=ilu_fill, ncomp=3 if elastic else 1,
                       mls_clip=args.mls_clip, dense_apply=nnms.INVERSE if xinv_mode else nnms.SWEEPS)
    t1 = time.perf_counter()
    load = W.ELASTIC_FORCE if elastic else 1.0

    def assemble(kappa):
        return nnms.System(h, kappa, load, poisson_ratio=W.ELASTIC_NU)

    s = assemble(pb.kappa)
    t2 = time.perf_counter()
    log(f"[bench] structure setup {t1 - t0:.2f} s, numeric setup (assembly + LU) {t2 - t1:.3f} s")
    from paper_2412_08981_amd import autotune
    tp = time.perf_counter()
    tuning = autotune.tune(s, cache=args.tuning_cache)
    log(f"[bench] launch shapes ({time.perf_counter() - tp:.2f} s): {tuning}")
    if args.factor_only:
        # the fine level's numeric factorisation alone (for counter runs)
        fb = 8 if prec == nnms.FP64 else 4
        msf = s.time_kernel(6, 0, reps=3)
        tf = lu_flops(h, 0) / (msf * 1e-3) / 1e12
        print(json.dumps({"factor_l0_launches": 1 + 3, "factor_l0_ms": msf, "factor_l0_flops": lu_flops(h, 0),
                          "factor_l0_TFLOPs": tf, "frac_of_mfma_peak": tf / MFMA_PEAK_TFLOPS[fb]}))
        return
    if args.transfers_only:
        # the transfers of every level at the tuned shapes (20 timed launches each)
        sb = 8 if prec == nnms.FP64 else 4
        out = {"workload": pb.name, "pt_lanes": tuning["pt_lanes"][:h.L - 1]}
        for lvl in range(h.L - 1):
            mst = s.time_kernel(3, lvl, reps=20)
            msp = s.time_kernel(2, lvl, reps=20)
            rb, pbytes = restrict_bytes(h, lvl, sb), prolong_bytes(h, lvl, sb)
            out.update({f"restrict_l{lvl}_launches": 1 + 20, f"restrict_l{lvl}_ms": mst,
                        f"restrict_l{lvl}_algorithmic_bytes": rb,
                        f"restrict_l{lvl}_frac_of_hbm_peak": rb / (mst * 1e-3) / HBM_PEAK_GBS / 1e9,
                        f"prolong_l{lvl}_launches": 1 + 20, f"prolong_l{lvl}_ms": msp,
                        f"prolong_l{lvl}_algorithmic_bytes": pbytes,
                        f"prolong_l{lvl}_frac_of_hbm_peak": pbytes / (msp * 1e-3) / HBM_PEAK_GBS / 1e9})
        print(json.dumps(out))
        return
    if args.kernels_only:
        # same launch shapes and repetition counts as the roofline figures below
        sb = 8 if prec == nnms.FP64 else 4
        fac_bytes = h.level_info(0).factor_elems * sb
        ms_copy = s.time_kernel(4, 0, reps=3)
        ms_read = s.time_kernel(5, 0, reps=5)
        ms_ras = s.time_kernel(0, 0, reps=10)
        out = {"copy_bytes": (fac_bytes // 16) * 16, "copy_launches": 1 + 3, "copy_ms": ms_copy,
               "read_launches": 1 + 5, "read_ms": ms_read,
               "ras_launches": 1 + 10, "ras_ms": ms_ras, "ras_algorithmic_bytes": smoother_bytes(h, 0, sb),
               "ras_hip_sha256_16": source_hash()}
        if h.L > 2 and h.level_info(1).subsolver != nnms.ILU:
            # the second level: its own copy reference and smoother launches
            fb1 = h.level_info(1).factor_elems * sb
            out.update({"l1_copy_bytes": (fb1 // 16) * 16, "l1_copy_ms": s.time_kernel(4, 1, reps=3),
                        "l1_ras_launches": 1 + 20, "l1_ras_ms": s.time_kernel(0, 1, reps=20),
                        "l1_ras_algorithmic_bytes": smoother_bytes(h, 1, sb)})
        print(json.dumps(out))
        return
    b = s.rhs()
    n0 = s.n[0]
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros(n0, dtype=torch.float64, device="cuda")
    graph = not args.no_graph
    infos = []
    for _ in range(args.warmup):
        infos.append(s.solve_device(bd.data_ptr(), xd.data_ptr(), graph=graph))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        info = s.solve_device(bd.data_ptr(), xd.data_ptr(), graph=graph)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    value = args.steps / el
    log(f"[bench] {args.steps} solves in {el:.3f} s: {info.iterations} iterations, relres {info.relres:.3e}")

    # the same solve through host buffers (b copied in, x copied out over PCIe):
    # reported beside the device-resident rate, never as the value
    b_host = np.ascontiguousarray(b)
    s.solve(b_host, graph=graph)
    th = time.perf_counter()
    nh = max(3, args.steps // 4)
    for _ in range(nh):
        s.solve(b_host, graph=graph)
    host_rate = nh / (time.perf_counter() - th)

    # numeric setup per parameter (assembly + extraction + LU), timed separately
    tp = time.perf_counter()
    s2 = assemble(W.kappa_draw(204, 999))
    torch.cuda.synchronize()
    t_assemble = time.perf_counter() - tp
    s2.destroy()

    # roofline of the dominant kernel: the fine-level smoother
    sb = 8 if prec == nnms.FP64 else 4
    ms = s.time_kernel(0, 0, reps=10)
    ach = smoother_bytes(h, 0, sb) / (ms * 1e-3) / 1e9
    extra = {}
    if not ilu_mode:
        fac_bytes = (h.level_info(0).factor_elems * sb // 16) * 16
        ms_read = s.time_kernel(5, 0, reps=5)
        extra["read_reference_GBs"] = round(fac_bytes / (ms_read * 1e-3) / 1e9, 1)
        extra["smoother_l0_frac_of_read_reference"] = round(ach / extra["read_reference_GBs"], 4)
    for lvl in range(h.L):
        extra[f"smoother_l{lvl}_ms"] = round(s.time_kernel(0, lvl, reps=10), 4)
    for lvl in range(h.L - 1):
        msr = s.time_kernel(1, lvl, reps=20)
        extra[f"residual_l{lvl}_ms"] = round(msr, 4)
        extra[f"residual_l{lvl}_GBs"] = round(spmv_bytes(h, lvl, sb) / (msr * 1e-3) / 1e9, 1)
        msp = s.time_kernel(2, lvl, reps=20)
        extra[f"prolong_l{lvl}_ms"] = round(msp, 4)
        extra[f"prolong_l{lvl}_GBs"] = round(prolong_bytes(h, lvl, sb) / (msp * 1e-3) / 1e9, 1)
        mst = s.time_kernel(3, lvl, reps=20)
        extra[f"restrict_l{lvl}_ms"] = round(mst, 4)
        extra[f"restrict_l{lvl}_GBs"] = round(restrict_bytes(h, lvl, sb) / (mst * 1e-3) / 1e9, 1)
    # numeric factorisation per level (fill + extraction + blocked LU) against the MFMA peak
    for lvl in range(h.L):
        fb = 8 if (prec == nnms.FP64 or lvl == h.L - 1) else 4
        msf = s.time_kernel(6, lvl, reps=3)
        extra[f"factor_l{lvl}_ms"] = round(msf, 3)
        if h.level_info(lvl).subsolver == nnms.ILU:
            continue  # ILU factorisation: level-scheduled, no dense flops to count
        tf = lu_flops(h, lvl) / (msf * 1e-3) / 1e12
        extra[f"factor_l{lvl}_TFLOPs"] = round(tf, 2)
        extra[f"factor_l{lvl}_frac_of_mfma_peak"] = round(tf / MFMA_PEAK_TFLOPS[fb], 4)
    extra["parametric_solves_per_s"] = round(1.0 / (t_assemble + el / args.steps), 3)
    extra["host_buffer_solves_per_s"] = round(host_rate, 3)
    log(f"[bench] kernels: {extra}")

    # the metric's other legs on the same problem and the batched instances
    legs = {}
    x_mixed = None
    if (not args.no_legs and not coarsened and args.precision == "fp64" and not mls_mode and not ilu_mode
            and not elastic and not args.nparts and args.workload == "cube48"):
        hm = nnms.Hierarchy(meshes, pb.nparts, overlap=pb.overlap, its=pb.its, precision=nnms.MIXED,
                            dense_apply=nnms.INVERSE if xinv_mode else nnms.SWEEPS)
        sm = nnms.System(hm, pb.kappa, 1.0)
        tm = autotune.tune(sm, cache=args.tuning_cache)
        xm = torch.zeros(n0, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            sm.solve_device(bd.data_ptr(), xm.data_ptr(), graph=graph)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            im = sm.solve_device(bd.data_ptr(), xm.data_ptr(), graph=graph)
        torch.cuda.synchronize()
        elm = time.perf_counter() - t
        x_mixed = xm.cpu().numpy()
        legs["mixed"] = {"workload": "the same 48^3/24^3/10^3 problem in mixed precision (FP32 subdomain factors, "
                                     "smoothing and transfers; FP64 FGMRES, Arnoldi and coarsest LU)",
                         "solves_per_s": round(args.steps / elm, 3), "ms_per_solve": round(1e3 * elm / args.steps, 3),
                         "iterations": im.iterations, "relres": im.relres,
                         "gain_over_fp64": round(el / elm, 3), "tuning": tm}
        log(f"[bench] mixed leg: {legs['mixed']}")
        sm.destroy()
        del hm
        b_r = batched_leg(args, 3)
        legs["batched"] = {"workload": f"{b_r['count']} parametric instances, fine n in {{24,32,40,48,64}}, "
                                       "3 non-nested levels each, mixed precision, one launch sequence per Arnoldi "
                                       "step for all (HIP graph)",
                           "solves_per_s": round(b_r["solves_per_s"], 3),
                           "sequential_solves_per_s": round(b_r["sequential_solves_per_s"], 3),
                           "batch_gain": round(b_r["solves_per_s"] / b_r["sequential_solves_per_s"], 3),
                           "max_relres": b_r["max_relres"], "iterations_max": max(b_r["iterations"]),
                           "batch_equals_alone_bitwise": b_r["bitwise_equal_alone"]}
        log(f"[bench] batched leg: {legs['batched']}")

    x = xd.cpu().numpy()
    out = {
        "metric": "solves/s to rel-res 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == nnms.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"P1 linear elasticity (three unknowns per vertex, field-split transfers), "
                                f"jittered unit cube, 3 non-nested levels 32^3/16^3/7^3 (35937 fine vertices, "
                                f"107811 unknowns), Young's modulus from the log-Gaussian field, Poisson's ratio "
                                f"{W.ELASTIC_NU}, body force {W.ELASTIC_FORCE}, " if elastic else
                                "jittered unit cube, 2 non-nested levels 16^3/6^3 (4913 fine vertices, 24576 tets), "
                                "kappa = 1, f = 1, " if args.workload == "cube16" else
                                f"jittered unit cube, 3 non-nested levels 96^3/48^3/20^3 "
                                f"({pb.meshes[0].nv} fine vertices), log-Gaussian kappa (8 centres), "
                                if args.workload == "served96" else
                                f"jittered unit cube, 3 non-nested levels 48^3/24^3/10^3 "
                                f"(117649 fine vertices, 663552 tets), log-Gaussian kappa (8 centres), ")
                               + f"{'+'.join(str(p) for p in pb.nparts)} subdomains overlap 1, FGMRES(30) to 1e-8, "
                               f"{args.precision}"
                               + (f", MLS transfer (scale {args.mls_alpha} x mean coarse edge"
                                  + (", neighbourhoods clipped to the target's subdomain)" if args.mls_clip else ")")
                                  if mls_mode else "")
                               + (f", ILU({args.ilu_fill}) subdomain solves" if ilu_mode else "")
                               + (", dense subdomain solves through inverse panels" if xinv_mode else "")
                               + (f", coarse levels by Algorithm 1 (rounds {rounds}; interior vertices "
                                  f"{[int((m.dirichlet == 0).sum()) for m in coarsened]})" if coarsened else ""),
                   "iterations": info.iterations, "relres": info.relres,
                   "numeric_setup_s": round(t_assemble, 4), "structure_setup_s": round(t1 - t0, 3),
                   "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": None if ilu_mode else load_traffic(args.precision,
                                                                   "k_xapply" if xinv_mode else "k_ras"),
                     "kernel": ("k_ilu_apply (fine-level ILU smoother)" if ilu_mode else
                                "k_xapply (fine-level smoother, inverse panels)" if xinv_mode else
                                "k_ras2 (fine-level smoother, two-block work items)" if tuning["ras_blocks"][0] == 2
                                else "k_ras (fine-level smoother)"), "ms": round(ms, 4)},
        "kernels": extra,
    }
    if legs:
        out["legs"] = legs
    if not args.no_cpu_baseline:
        pb_o = pb
        if coarsened:
            # the oracle coarsens the fine mesh itself (equal to the library's, bit for bit)
            from oracle import coarsen as ocoarsen
            om = [fine_mesh]
            for l in range(1, len(coarsened)):
                r = ocoarsen.coarsen(om[-1].xyz, om[-1].tets, om[-1].dirichlet, rounds[l - 1], l)
                om.append(W.Mesh(r.xyz, r.tets.astype(np.int32), r.dirichlet, 0))
            pb_o = W.Problem(pb.name, om, pb.nparts, pb.kappa, precision=pb.precision)
        cb, oh, ores = cpu_baseline(pb_o, mls_alpha=args.mls_alpha if mls_mode else None, elasticity=elastic,
                                    mls_clip=args.mls_clip)
        out["cpu_baseline"] = cb
        from oracle import problem as oprob  # the oracle's own x* for the error report
        xs = ores.x
        out["config"]["rel_err_vs_oracle_fgmres"] = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
        out["config"]["oracle_iterations"] = ores.iterations
        if x_mixed is not None:
            legs["mixed"]["rel_err_vs_oracle_fgmres"] = float(np.linalg.norm(x_mixed - xs) / np.linalg.norm(xs))
        if legs:
            cb["other_workloads"] = cpu_baseline_extra()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
