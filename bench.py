#!/usr/bin/env python3
"""Benchmark of the multigrid hot path on one MI355X.

Workload (default): 3D Poisson, LDG Q_3 (64 unknowns per element, Legendre
basis), uniform 64^3 grid of the unit cube (16,777,216 unknowns), Dirichlet
boundaries, seeded N(0,1) right-hand sides; SAI_1 (OI ordering) V-cycle with
FP32 block storage (operators; the SAI matrices optionally in BF16), its block
products in FP64 or (ldgmg_fp32_products) in FP32 on the matrix cores, as the
preconditioner of FP64 CG, solved to a 1e-10 relative residual.  One step = one full solve from x0 = 0 (every stage of the path:
residuals, SAI applies, transfers, bottom solve, V-cycle control, CG).  Inputs
are resident in HBM before the timed region.

Printed JSON (one line on stdout):
  value        V-cycle DOF/s = fine unknowns x V-cycles in the timed solves / time,
               of the fastest path (FP32 or BF16-SAI storage, FP64 or FP32
               products) that needs exactly the CG iterations of FP32 storage
               with FP64 products and meets the residual bar
  solves_per_s, p50_ms / p99_ms per solve, iterations, eta, true residual
  fp32_path, bf16s_path, fp64_path   the same solves per storage precision (same MI355X)
  fp32p_path, bf16sp_path            the FP32 and BF16-SAI handles with FP32 products
  expanded_path the headline precision with every block stored per slot (streamed from HBM)
  roofline     the dominant kernel (forward BSR apply with FP32 blocks on the
               fine level), timed with HIP events inside the library over the
               timed region; algorithmic bytes per launch / mean duration
  cpu_baseline the CPU oracle timed on this host on a bounded sample
Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "V-cycle DOF/s & solves/s to 1e-10 rel. residual (FP32 vs FP64); p50/p99 ms"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TF = 78.6      # MI355X FP64 vector (FMA) peak
FP64_MFMA_PEAK_TF = 78.6        # MI355X dense FP64 matrix-core peak
FP32_MFMA_PEAK_TF = 157.3       # MI355X dense FP32 matrix-core peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def run_path(L, torch, args, precision, rhs, prof, storage="auto", fp32_products=()):
    """Set up one precision and device storage, warm up, time args.steps
    solves.  Returns stats; for each entry of fp32_products (a name) the same
    handle is timed again with ldgmg_fp32_products on, and those stats are
    returned under that name."""
    t0 = time.time()
    s = L.Solver(dim=3, n=args.n, p=args.p, smoother="sai", sai_level=1, order="OI",
                 precision=precision, storage=storage)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"[{precision}] setup {setup_s:.1f}s ndofs {s.ndofs} levels {s.nlevels}")
    out = time_solves(L, torch, args, s, precision, precision, rhs, prof, setup_s, False)
    for name in fp32_products:
        L.ldgmg_fp32_products(s.handle, True)
        out[name] = time_solves(L, torch, args, s, precision, name, rhs, prof, setup_s, True)
        L.ldgmg_fp32_products(s.handle, False)
    s.close()
    torch.cuda.synchronize()
    return out


def time_solves(L, torch, args, s, precision, label, rhs, prof, setup_s, fp32_products, krylov="cg",
                maxit=200, steps=None, warmup=None):
    """Warm up and time `steps` (default args.steps) solves on handle s
    (storage precision `precision`, logged as `label`)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    x = torch.empty_like(rhs[0])
    for i in range(warmup):
        info = s.solve(rhs[i], x, krylov, 1e-10, maxit)
        log(f"[{label}] warmup {i}: iters {info['iters']}")
    stream = torch.cuda.current_stream()
    if prof:
        L.ldgmg_profile(s.handle, True)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    infos = []
    t0 = time.time()
    for k in range(steps):
        b = rhs[warmup + k]
        ev[k][0].record(stream)
        info = s.solve(b, x, krylov, 1e-10, maxit, stream=stream)
        ev[k][1].record(stream)
        infos.append(info)
        log(f"[{label}] step {k}: iters {info['iters']} rel_res {info['rel_res_true']:.2e}")
    torch.cuda.synchronize()
    wall = time.time() - t0
    lat = [a.elapsed_time(b) for a, b in ev]
    total_ms = ev[0][0].elapsed_time(ev[-1][1])
    vcycles = sum(i["vcycles"] for i in infos)
    out = {
        "setup_s": setup_s,
        "total_ms": total_ms,
        "wall_s": wall,
        "ms_per_solve": total_ms / steps,
        "solves_per_s": 1000.0 * steps / total_ms,
        "vcycle_dof_per_s": s.ndofs * vcycles / (total_ms / 1000.0),
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "iters": [i["iters"] for i in infos],
        "converged": all(i["converged"] for i in infos),
        "eta": float(sum(i["eta"] for i in infos) / len(infos)),
        "rel_res_true_max": max(i["rel_res_true"] for i in infos),
        "vcycles": vcycles,
        "ndofs": s.ndofs,
        "fp32_products": fp32_products,
    }
    if prof:
        info0 = L.ldgmg_level_info(s.handle, 0)
        bs = s.bs
        N = s.ndofs
        ne = info0["nelem"]
        # bytes per stored entry: operators A, smoother B (and its transposed copy)
        eb_a = 8 if precision == "fp64" else 4
        eb_s = {"fp64": 8, "fp32": 4, "bf16s": 2}[precision]
        storage = L.ldgmg_level_storage(s.handle, 0)
        kinds = {}
        for kind in ("A", "S", "ST", "A64"):
            cnt, ms = L.ldgmg_profile_read(s.handle, kind)
            if kind != "A" and not cnt:
                continue
            nnzb = info0["nnzb_A"] if kind in ("A", "A64") else info0["nnzb_S"]
            ebk = 8 if kind == "A64" else eb_a if kind == "A" else eb_s
            pool = storage["pool_A"] if kind in ("A", "A64") else storage["pool_S"]
            tiled = storage["tiled_A"] if kind in ("A", "A64") else storage["tiled_S"]
            # algorithmic HBM bytes per launch: the stored blocks (expanded: every
            # slot's block; pooled: the distinct blocks once plus a 4-byte block
            # id per slot) + block indices + vectors (input read, added vector
            # read, output written; FP64, but FP32 for the smoothing residual
            # with FP32 products)
            vec = 3 * N * 8 if kind != "A64" else 2 * N * 8
            if fp32_products and tiled and bs % 16 == 0 and storage["tiled_A"] and storage["tiled_S"]:
                # the smoothing vectors are FP32 where they are only operands:
                # B and B^T read r in FP32, read and write x in FP64 and write
                # its FP32 copy; the A launches read that copy and b (FP64), and
                # of the 6 fine A launches of a V-cycle (nu1 = nu2 = 3, x = 0 at
                # entry) 5 write r in FP32 and the one before restriction in FP64
                vec = (4 + 8 + 8 + 4) * N if kind in ("S", "ST") else \
                    ((5 * (4 + 8 + 4) + (4 + 8 + 8)) * N) // 6 if kind == "A" else vec
            idx = (ne + 1) * 4 + nnzb * 4
            blocks = pool * bs * bs * ebk + nnzb * 4 if pool else nnzb * bs * bs * ebk
            byts = blocks + idx + vec
            flops = 2 * nnzb * bs * bs          # one FMA per stored entry (FP64 or FP32 products)
            mean_s = ms / cnt / 1e3 if cnt else None
            kinds[kind] = {"count": cnt, "ms_total": ms, "bytes_per_launch": byts, "flops_per_launch": flops,
                           "pooled": bool(pool), "tiled": bool(tiled), "mean_ms": ms / cnt if cnt else None,
                           "gbs": byts / mean_s / 1e9 if cnt else None,
                           "tflops": flops / mean_s / 1e12 if cnt else None}
        out["kernels"] = kinds
        out["storage"] = storage
        L.ldgmg_profile(s.handle, False)
    return out


def kernel_source(kernel):
    """Code of a kernel family in kernels.hip (what the counter summaries are
    keyed on): the forward kernels (k_bsr_fwd and its multi-right-hand-side
    form) or the tiled kernel with its layout helpers, with // comments,
    trailing blanks and empty lines removed (edits of comments alone keep the
    key)."""
    src = open(os.path.join(ROOT, "paper_2412_12506_amd", "csrc", "kernels.hip")).read()
    sep = "// ---------------------------------------------------------------------------\n"
    if kernel == "tiled":
        a = src.index(sep + "// tiled forward BSR kernel")
        b = src.index("// generic BSR kernel for any block size")
    else:
        a = src.rindex("template <", 0, src.index("void k_bsr_fwd("))
        b = src.index(sep + "// transposed BSR kernel")
    lines = (line.split("//", 1)[0].rstrip() for line in src[a:b].splitlines())
    return "\n".join(line for line in lines if line) + "\n"


def counter_traffic(storage="expanded"):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if that summary was taken with the current kernel source
    (None otherwise)."""
    import hashlib
    name = {"expanded": "bsr_fwd_fp32_bs64", "pooled": "bsr_fwd_fp32_pooled_bs64",
            "tiled": "bsr_tiled_fp32_bs64", "tiled32": "bsr_tiled_fp32p_bs64"}[storage]
    prof = os.path.join(ROOT, "profiles", f"{name}_poisson3d_n64_counters.json")
    try:
        rec = json.load(open(prof))
        text = kernel_source("tiled" if storage.startswith("tiled") else "fwd")
        if hashlib.sha256(text.encode()).hexdigest()[:16] != rec["kernel_source_sha256_16"]:
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(n_cpu, min_seconds=10.0):
    """The oracle, as it stands, on a bounded sample of the same workload:
    3D Poisson Q_3, SAI_1 OI V-cycle in CG, on an n_cpu^3 grid (setup untimed;
    full CG solves of seeded right-hand sides timed until at least
    min_seconds of one-core work, at least two and at most 30 solves)."""
    from oracle import solver as osolver
    from ldg_inputs import rhs_normal
    t0 = time.time()
    lv, vc = osolver.build(3, n_cpu, 3)
    log(f"[cpu] oracle setup {time.time() - t0:.1f}s")
    ndofs = lv[0].A.shape[0]
    from threadpoolctl import threadpool_limits
    times, vcycles, iters = [], [], []
    with threadpool_limits(limits=1):       # the oracle's products run on one core
        while len(times) < 30 and (len(times) < 2 or sum(times) < min_seconds):
            b = rhs_normal(ndofs, len(times))
            t0 = time.time()
            r = osolver.solve(lv, vc, b, "cg")
            times.append(time.time() - t0)
            iters.append(r.iters)
            vcycles.append(r.iters + 1 - (1 if r.converged else 0))
    dt = sum(times)
    its = f"{min(iters)}" if min(iters) == max(iters) else f"{min(iters)}-{max(iters)}"
    return {"value": ndofs * sum(vcycles) / dt, "unit": "DOF/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{len(times)} FP64 CG solves (to 1e-10, {its} iterations each, {sum(vcycles)} V-cycles "
                       f"in all; right-hand-side seeds 0..{len(times) - 1}) of the same workload on a "
                       f"{n_cpu}^3 grid ({ndofs} unknowns), {dt:.1f} s on one host thread (BLAS limited to 1); "
                       f"setup untimed"),
            "seconds": dt, "solves_per_s": len(times) / dt, "host_cpus": os.cpu_count()}


# request catalogues of the serving workload: "full" is the mixed stream of
# 2D/3D Poisson and box-interface problems (2D 32^2..256^2, 3D 16^3..48^3,
# p = 1..3, contrast 1..1e4); "lite" keeps its 2D part and the 3D grids up to
# 32^3 with p <= 2
CATALOGUES = {
    "full": dict(grids2d=(32, 64, 128, 256), grids3d=(16, 24, 32, 48), degrees=(1, 2, 3),
                 contrasts=(1.0, 10.0, 1e2, 1e3, 1e4)),
    "lite": dict(grids2d=(32, 64, 128, 256), grids3d=(16, 24, 32), degrees=(1, 2),
                 contrasts=(1.0, 10.0, 1e2, 1e3, 1e4)),
}


def run_serving(args, torch, nested=False):
    """Replay the seeded request stream through the serving engine; one JSON
    line with solves/s and p50/p99 latency (arrival to completion).  nested:
    the reduced replay of the main line (the lite catalogue, --replay-requests
    requests), returned instead of printed."""
    from ldg_inputs import serving_requests
    from paper_2412_12506_amd.serving import ServingEngine, problem_key, summarize
    catalogue = "lite" if nested else args.serving_catalogue
    cat = CATALOGUES[catalogue]
    reqs = serving_requests(count=args.replay_requests if nested else args.serving_requests, **cat)
    free, total = torch.cuda.mem_get_info()
    budget = int(args.serving_budget_gib * (1 << 30)) if args.serving_budget_gib else int(free * 0.9)
    keys = sorted({problem_key(r) for r in reqs})
    setup_cmp = None
    if nested:
        # cache-miss cost: the host tier of the replay's keys built with the SAI
        # least-squares problems solved on the host, then on the GPU
        setup_cmp = {}
        for dev in (False, True):
            e2 = ServingEngine(budget, workers=args.serving_workers, setup_device=dev)
            setup_cmp["gpu" if dev else "host"] = e2.prebuild(keys, threads=4)
            e2.close()
        log(f"[serving] host tier: SAI solves on the host {setup_cmp['host']:.1f} s, on the GPU {setup_cmp['gpu']:.1f} s")
    eng = ServingEngine(budget, workers=args.serving_workers, setup_device=args.serving_setup_device or nested)
    log(f"[serving] {len(reqs)} requests, {len(keys)} hierarchies, budget {budget / 2**30:.1f} GiB")
    setup_s = eng.prebuild(keys, threads=4)
    log(f"[serving] host tier built in {setup_s:.1f} s")
    out = {}

    def replay(mode, scale):
        for e in eng.entries.values():          # every replay starts with an empty device tier
            if e.resident:
                e.solver.unload()
                e.resident, e.bytes = False, 0
        eng.used, eng.peak_used = 0, 0
        eng.results, eng.evictions, eng.admissions = [], [], []
        res = eng.run(reqs, time_scale=scale)
        for r in res:
            if not r.converged:
                log(f"[serving] {mode}: request {r.rid} {r.key} not converged: iters {r.iters} "
                    f"res {r.rel_res_true:.2e} batch {r.batch} {r.error}")
        st = summarize(res)
        st["uploads"] = len(eng.admissions)
        st["evictions"] = len(eng.evictions)
        st["peak_hbm_gib"] = eng.peak_used / 2 ** 30
        st["dof_per_s"] = st["dofs_solved"] / st["wall_s"] if st["wall_s"] else None
        out[mode] = st
        log(f"[serving] {mode}: {st}")

    # capacity: every request queued at once; then the stream at its arrival
    # times, scaled to the requested rate (0: 70% of the measured capacity)
    replay("saturated", 0.0)
    rate = args.serving_rate or 0.7 * out["saturated"]["solves_per_s"]
    base = len(reqs) / reqs[-1].arrival
    replay("offered", base / rate)
    out["offered"]["rate_per_s"] = rate
    eng.close()
    sat = out["saturated"]
    line = {
        "metric": METRIC, "value": sat["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": sat["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "block_storage": "f32", "data": "synthetic",
        "config": {"workload": f"serving_{len(reqs)}_mixed_{catalogue}",
                   "requests": len(reqs), "hierarchies": len(keys),
                   "offered_rate_per_s": out["offered"]["rate_per_s"],
                   "rtol": 1e-10, "smoother": "SAI_1 OI",
                   "outer": f"FP64 CG, continuous batching (ldgmg_solve_stream, {eng.max_batch} slots)",
                   "workers": args.serving_workers, "hbm_budget_gib": budget / 2 ** 30},
        "p50_ms": out["offered"]["p50_ms"], "p99_ms": out["offered"]["p99_ms"],
        "offered": out["offered"], "saturated": sat, "host_setup_s": setup_s,
        "host_tier_build_s": setup_cmp,
    }
    if nested:
        return {k: line[k] for k in ("value", "unit", "config", "p50_ms", "p99_ms", "offered", "saturated",
                                     "host_setup_s", "host_tier_build_s")}
    print(json.dumps(line), flush=True)


def kernel_summary(kinds, kind):
    v = kinds.get(kind)
    if not v or not v["count"]:
        return None
    return {kk: v[kk] for kk in ("count", "mean_ms", "gbs", "tflops", "bytes_per_launch", "flops_per_launch",
                                 "pooled", "tiled")}


def run_interface_config(L, torch, args, BASE_SEED):
    """96^3 elliptic interface, Q_2, viscosity 1e4 inside the sphere r = 0.3
    (element-centre test), FP32 storage, FP64 CG to 1e-10.  The coloured
    Gauss-Seidel OI V-cycle converges and is timed; the SAI_1 OI V-cycle does
    not converge on this curved interface (Section 3 of the design notes): it
    runs a bounded number of iterations, which times its fine-level B applies
    (expanded storage: the distinct columns of a curved interface are too many
    to pool), the HBM-bound kernel of this workload."""
    from ldg_inputs import mu_field, rhs_normal
    n, p = args.cfg3_n, 2
    mu = mu_field(3, n, "sphere", 0.3, 1e4)
    ndofs = n ** 3 * (p + 1) ** 3
    rhs = [torch.from_numpy(rhs_normal(ndofs, BASE_SEED + i)).cuda() for i in range(2)]
    out = {"workload": f"interface3d_p2_n{n}_sphere1e4", "fine_dofs": ndofs}
    for sm, label, maxit, steps, warm in (("gs", "gs_oi", 200, 1, 1), ("sai", "sai1_oi", args.cfg3_sai_maxit, 1, 0)):
        t0 = time.time()
        sv = L.Solver(dim=3, n=n, p=p, mu=mu, smoother=sm, sai_level=1, order="OI", precision="fp32")
        torch.cuda.synchronize()
        setup = time.time() - t0
        log(f"[interface {label}] setup {setup:.1f}s")
        r = time_solves(L, torch, args, sv, "fp32", f"interface {label}", rhs, True, setup, False,
                        maxit=maxit, steps=steps, warmup=warm)
        st = L.ldgmg_level_storage(sv.handle, 0)
        sv.close()
        keep = ("setup_s", "ms_per_solve", "solves_per_s", "vcycle_dof_per_s", "iters", "converged",
                "rel_res_true_max", "eta")
        out[label] = {k: r[k] for k in keep}
        out[label]["fine_storage"] = st
        out[label]["kernels"] = {kk: kernel_summary(r["kernels"], kk) for kk in ("A", "S", "ST", "A64")}
    b = out["sai1_oi"]["kernels"].get("S")
    if b and not b["pooled"]:
        out["roofline"] = {"bound": "hbm", "kernel": "k_bsr_fwd<fp32 blocks, fp64 vectors, bs=27, expanded> "
                                                     "(fine-level SAI_1 B apply)",
                           "achieved": b["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": b["gbs"] / HBM_PEAK_GBS, "traffic": None, "mean_ms": b["mean_ms"],
                           "bytes_per_launch": b["bytes_per_launch"]}
    return out


def run_stokes_config(L, torch, args, BASE_SEED):
    """256^2 multiphase stress-form Stokes, Q_2, viscosity 1e3 inside the disc
    r = 0.25, velocity Dirichlet, balanced SAI_1 OO V-cycle in FP64 left GMRES
    to ||V r|| <= 1e-10 ||V b||, FP32 storage; seeded N(0,1) body force."""
    from ldg_inputs import mu_field, stokes_body_force
    n, p = args.cfg4_n, 2
    mu = mu_field(2, n, "disc", 0.25, 1e3)
    rhs = [torch.from_numpy(stokes_body_force(2, n, 9, BASE_SEED + i)).cuda() for i in range(3)]
    t0 = time.time()
    sv = L.Solver(dim=2, n=n, p=p, system="stokes", gamma=1, mu=mu, smoother="sai", sai_level=1, order="OO",
                  precision="fp32")
    torch.cuda.synchronize()
    setup = time.time() - t0
    log(f"[stokes] setup {setup:.1f}s")
    r = time_solves(L, torch, args, sv, "fp32", "stokes sai1_oo", rhs, True, setup, False, krylov="gmres",
                    maxit=200, steps=2, warmup=1)
    st = L.ldgmg_level_storage(sv.handle, 0)
    nker = L.ldgmg_kernel(sv.handle)
    sv.close()
    keep = ("setup_s", "ms_per_solve", "solves_per_s", "vcycle_dof_per_s", "iters", "converged",
            "rel_res_true_max", "eta", "p50_ms", "p99_ms")
    out = {"workload": f"stokes2d_stress_p2_n{n}_disc1e3", "fine_dofs": sv.ndofs, "krylov": "left GMRES",
           "smoother": "SAI_1 OO", "kernel_dim": nker, **{k: r[k] for k in keep}}
    out["fine_storage"] = st
    out["kernels"] = {kk: kernel_summary(r["kernels"], kk) for kk in ("A", "S", "ST", "A64")}
    a = out["kernels"]["A"]
    if a:
        if a["tiled"] or a["pooled"]:
            out["roofline"] = {"bound": "mfma" if a["tiled"] else "alu", "kernel": "fine-level A apply (bs=27)",
                               "achieved": a["tflops"], "peak": FP64_MFMA_PEAK_TF, "unit": "TFLOP/s",
                               "frac": a["tflops"] / FP64_MFMA_PEAK_TF, "traffic": None, "mean_ms": a["mean_ms"]}
        else:
            out["roofline"] = {"bound": "hbm", "kernel": "fine-level A apply (bs=27, expanded)",
                               "achieved": a["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": a["gbs"] / HBM_PEAK_GBS, "traffic": None, "mean_ms": a["mean_ms"]}
    return out


def run_batched(L, torch, args, BASE_SEED):
    """Batched CG of K right-hand sides on one hierarchy (the serving step):
    3D Poisson Q_p on n^3, SAI_1 OI, BF16-SAI tiled storage (the batched
    products on the matrix cores, (row, right-hand side) pairs as MFMA
    columns), FP64 products.  One JSON line: V-cycle DOF/s over the batch,
    ms per batch, iterations per right-hand side, and the same K right-hand
    sides solved one at a time for comparison."""
    from ldg_inputs import rhs_normal
    k = args.batch_k
    s = L.Solver(dim=3, n=args.n, p=args.p, smoother="sai", sai_level=1, order="OI", precision="bf16s",
                 storage="tiled")
    bs = [torch.from_numpy(rhs_normal(s.ndofs, BASE_SEED + q)).cuda() for q in range(k)]
    xs = [torch.empty_like(b) for b in bs]
    L.ldgmg_solve_batch(s.handle, bs, xs)                   # warm-up (allocates the batch workspace)
    torch.cuda.synchronize()
    times, infos = [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        infos = L.ldgmg_solve_batch(s.handle, bs, xs)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[batch k={k}] {times[-1] * 1e3:.1f} ms, iters {[i['iters'] for i in infos]}")
    single = []
    for q in range(k):
        t0 = time.perf_counter()
        s.solve(bs[q], xs[q])
        torch.cuda.synchronize()
        single.append(time.perf_counter() - t0)
    import numpy as np
    t = float(np.median(times))
    vc = sum(i["vcycles"] for i in infos)
    line = {"metric": "batched V-cycle DOF/s (serving step)", "value": s.ndofs * vc / t, "unit": "DOF/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t * 1e3, "higher_is_better": True,
            "dtype": "f64", "block_storage": "A f32, SAI B bf16, tiled", "data": "synthetic",
            "config": {"workload": f"poisson3d_p{args.p}_n{args.n}_sai1_oi_cg_batch{k}", "k": k,
                       "fine_dofs": s.ndofs},
            "iters": [i["iters"] for i in infos], "single_solve_ms_sum": sum(single) * 1e3,
            "speedup_vs_single": sum(single) / t}
    s.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="grid size per side")
    ap.add_argument("--p", type=int, default=3, help="polynomial degree")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-storage comparison")
    ap.add_argument("--no-bf16s", action="store_true", help="skip the BF16 SAI-storage path")
    ap.add_argument("--no-fp32-storage", action="store_true",
                    help="skip the FP32-storage path (e.g. to count one path's kernels alone)")
    ap.add_argument("--no-expanded", action="store_true", help="skip the expanded-storage reference path")
    ap.add_argument("--no-fp32-products", action="store_true",
                    help="skip the FP32-product timings (ldgmg_fp32_products) of the FP32 and BF16-SAI paths")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=8, help="grid of the CPU oracle sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--serving", action="store_true",
                    help="run the serving workload instead (a separate JSON line)")
    ap.add_argument("--serving-catalogue", choices=sorted(CATALOGUES), default="full")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="mean arrivals per second of the offered replay (0: 70%% of the saturated throughput)")
    ap.add_argument("--serving-workers", type=int, default=4)
    ap.add_argument("--serving-budget-gib", type=float, default=0.0, help="0: 90%% of free HBM")
    ap.add_argument("--serving-setup-device", action="store_true",
                    help="solve the SAI least-squares problems of cache misses on the GPU")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the interface (96^3) and Stokes (256^2) workloads nested in the line")
    ap.add_argument("--cfg3-n", type=int, default=96, help="grid of the interface workload")
    ap.add_argument("--cfg3-sai-maxit", type=int, default=30,
                    help="CG iterations of the (non-converging) SAI_1 run of the interface workload")
    ap.add_argument("--cfg4-n", type=int, default=256, help="grid of the Stokes workload")
    ap.add_argument("--no-serving-replay", action="store_true",
                    help="skip the reduced serving replay nested in the line")
    ap.add_argument("--replay-requests", type=int, default=96, help="requests of the nested serving replay")
    ap.add_argument("--batch-k", type=int, default=0, metavar="K",
                    help="only time batched CG (ldgmg_solve_batch) of K right-hand sides on the --n / --p "
                         "Poisson workload, BF16-SAI tiled storage (a separate JSON line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU path is not part of this build "
              "(see DESIGN.md, 'How the path would shard').", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes BYTES each, so the
        # HBM counters of this dispatch give the scale for the solver's kernels
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 3}), flush=True)
        return
    from paper_2412_12506_amd import ldgmg as L
    from ldg_inputs import rhs_normal, BASE_SEED

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serving:
        run_serving(args, torch)
        return
    if args.batch_k:
        run_batched(L, torch, args, BASE_SEED)
        return
    ndofs = args.n ** 3 * (args.p + 1) ** 3
    nrhs = args.warmup + args.steps
    rhs = [torch.from_numpy(rhs_normal(ndofs, BASE_SEED + i)).to(dev) for i in range(nrhs)]
    torch.cuda.synchronize()
    paths = {}
    for prec in (() if args.no_fp32_storage else ("fp32",)) + (() if args.no_bf16s else ("bf16s",)):
        pname = prec + "p"                  # the same handle with FP32 products
        r = run_path(L, torch, args, prec, rhs, prof=True, fp32_products=() if args.no_fp32_products else (pname,))
        if pname in r:
            paths[pname] = r.pop(pname)
        paths[prec] = r
    fp64 = None if args.no_fp64 else run_path(L, torch, args, "fp64", rhs, prof=False)
    # streaming reference: the same solves with every block stored per slot
    expanded = None if args.no_expanded else run_path(L, torch, args, "bf16s" if "bf16s" in paths else "fp32",
                                                      rhs, prof=True, storage="expanded")
    del rhs
    cfg3 = cfg4 = replay = None
    if not args.no_configs:
        cfg3 = run_interface_config(L, torch, args, BASE_SEED)
        cfg4 = run_stokes_config(L, torch, args, BASE_SEED)
    if not args.no_serving_replay:
        replay = run_serving(args, torch, nested=True)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_n)

    # headline path: the fastest of FP32 / BF16-SAI storage, each with FP64 or
    # FP32 products, among those that need exactly the CG iterations of FP32
    # storage with FP64 products on every right-hand side and reach the same
    # true FP64 residual bar
    ref = "fp32" if "fp32" in paths else next(iter(paths))
    ref_iters = paths[ref]["iters"]
    ok = [nm for nm, pth in paths.items() if pth["iters"] == ref_iters and pth["rel_res_true_max"] <= 2e-10]
    head = max(ok or [ref], key=lambda nm: paths[nm]["vcycle_dof_per_s"])
    hp = paths[head]
    k = hp["kernels"]
    p32 = hp["fp32_products"]
    bf = paths.get("bf16s")
    # dominant kernel: the fine-level forward BSR apply of A with FP32 blocks
    # (with FP32 smoother storage the B applies run the same instantiation)
    dom = ("A", "S") if head.startswith("fp32") and \
        (k["A"]["pooled"], k["A"]["tiled"]) == (k["S"]["pooled"], k["S"]["tiled"]) else ("A",)
    cnt = sum(k[d]["count"] for d in dom)
    ms = sum(k[d]["ms_total"] for d in dom)
    byts = sum(k[d]["bytes_per_launch"] * k[d]["count"] for d in dom) / max(cnt, 1)
    flops = sum(k[d]["flops_per_launch"] * k[d]["count"] for d in dom) / max(cnt, 1)
    mean_s = ms / max(cnt, 1) / 1000.0
    pooled, tiled = k["A"]["pooled"], k["A"]["tiled"]
    name = f"k_bsr_fwd<fp32 blocks, fp64 vectors, bs=64, {'pooled' if pooled else 'expanded'}> (fine level)"
    if tiled:
        # pooled blocks applied on the matrix cores: priced against the dense
        # MFMA peak of the product type (2 flops per stored entry and row)
        if p32:
            name = "k_bsr_tiled<fp32 blocks, bs=64, FP32 products> (fine level, v_mfma_f32_16x16x4f32)"
            peak = FP32_MFMA_PEAK_TF
        else:
            name = "k_bsr_tiled<fp32 blocks, bs=64> (fine level, v_mfma_f64_16x16x4f64)"
            peak = FP64_MFMA_PEAK_TF
        achieved = flops / mean_s / 1e12 if cnt else None
        roof = {"bound": "mfma", "kernel": name, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak if achieved else None,
                "traffic": counter_traffic("tiled32" if p32 else "tiled"),
                "hbm_gbs": byts / mean_s / 1e9 if cnt else None, "flops_per_launch": flops}
    elif pooled:
        # blocks come from the caches; each stored entry costs a widening and an
        # FP64 FMA on the vector ALUs: priced against the FP64 vector peak
        achieved = flops / mean_s / 1e12 if cnt else None
        roof = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": FP64_VECTOR_PEAK_TF,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TF if achieved else None,
                "traffic": counter_traffic("pooled"), "hbm_gbs": byts / mean_s / 1e9 if cnt else None,
                "flops_per_launch": flops}
    else:
        achieved = byts / mean_s / 1e9 if cnt else None
        roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": counter_traffic("expanded")}
    roof.update({"launches": cnt, "mean_ms": ms / max(cnt, 1), "bytes_per_launch": byts,
                 "other_kernels": {kk: {"mean_ms": v["mean_ms"], "gbs": v["gbs"], "tflops": v["tflops"],
                                        "count": v["count"], "pooled": v["pooled"], "tiled": v["tiled"],
                                        "bytes_per_launch": v["bytes_per_launch"]}
                                   for kk, v in k.items() if kk not in dom}})
    summary = ("vcycle_dof_per_s", "solves_per_s", "ms_per_solve", "p50_ms", "p99_ms", "iters",
               "rel_res_true_max", "setup_s")
    line = {
        "metric": METRIC,
        "value": hp["vcycle_dof_per_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hp["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p32 else "f64",
        "dtype_detail": ("block products f32 on the matrix cores (V-cycle applies); vectors, transfers, "
                         "bottom and CG f64" if p32 else "f64 arithmetic on f32/bf16-stored blocks"),
        "headline_path": head,
        "block_storage": ("A f32, SAI B bf16" if head.startswith("bf16s") else "f32")
                         + (", tiled" if k["A"]["tiled"] else ", pooled" if k["A"]["pooled"] else ", expanded"),
        "data": "synthetic",
        "config": {"workload": f"poisson3d_p{args.p}_n{args.n}_sai1_oi_cg",
                   "fine_dofs": ndofs, "rtol": 1e-10, "rhs": "N(0,1) seeded",
                   "smoother": "SAI_1 OI, nu1=nu2=3", "outer": "FP64 CG"},
        "solves_per_s": hp["solves_per_s"],
        "p50_ms": hp["p50_ms"],
        "p99_ms": hp["p99_ms"],
        "iters": hp["iters"],
        "eta": hp["eta"],
        "rel_res_true_max": hp["rel_res_true_max"],
        "setup_s": hp["setup_s"],
        "fp32_path": {k2: paths["fp32"][k2] for k2 in summary} if "fp32" in paths else None,
        "bf16s_path": None if bf is None else {k2: bf[k2] for k2 in summary},
        "fp32p_path": {k2: paths["fp32p"][k2] for k2 in summary} if "fp32p" in paths else None,
        "bf16sp_path": {k2: paths["bf16sp"][k2] for k2 in summary} if "bf16sp" in paths else None,
        "fp64_path": None if fp64 is None else {k2: fp64[k2] for k2 in summary},
        "expanded_path": None if expanded is None else dict(
            {k2: expanded[k2] for k2 in summary},
            dominant_kernel={kk: expanded["kernels"]["A"][kk] for kk in ("mean_ms", "gbs", "bytes_per_launch")},
            frac_hbm=expanded["kernels"]["A"]["gbs"] / HBM_PEAK_GBS if expanded["kernels"]["A"]["gbs"] else None),
        "roofline": roof,
        "cpu_baseline": cpu,
        "interface_path": cfg3,
        "stokes_path": cfg4,
        "serving_replay": replay,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
