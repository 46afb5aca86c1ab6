"""Benchmark of the Symanzik gauge force on one MI355X.

Workload: the 32^3x64 periodic lattice with near-thermal links U = exp(i 0.25 r.T)
(r ~ N(0,1), seed 2), u0 = 0.8677, beta = 3. One step is one force pass over all
8,388,608 links with the action fused (coefficients, staple sums, TA force, FP64
action reduction), on fields resident in HBM in the even-odd SoA layout. The
headline is FP32 link products with FP64 action; the FP64 form is timed beside it.

Prints one JSON line (metric, value = link-forces/s, roofline of the dominant kernel,
CPU-oracle baseline, errors of the FP32 and FP64 forces and actions against the FP64
oracle on every link, FP64 timing, leapfrog step timing and the other rows).

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --copy-calibration      # plain copy kernel for rocprof byte counters
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "link-forces/sec + % HBM/VALU roofline, Symanzik force 32^3x64, FP32 vs FP64"
WORKLOAD = "thermal_32x32x32x64"

# Work per link-force (flop; FMA = 2; SU(3) product 198, product accumulated into a
# matrix 216), each figure stated beside its constant.
FLOP_PAPER = 36770          # the paper's algorithm: 180 staple products, sums, U t, TA
FLOP_STAPLES = 2079         # factored pass 1: 42 products per site (10.5 per link)
FLOP_FACTORED = 12909       # factored pass 2: 57 products, 55 accumulations, weights, traces, TA
FLOP_DIRECT = 36940         # direct kernel: 181 products + sums, traces, TA
# Minimum HBM bytes per link of each kernel (read once / write once), per real size r.
BYTES_STAPLES = lambda r: (12 + 6 * 12) * r              # read U (two rows), write 6 two-row staples
BYTES_FACTORED = lambda r: (12 + 6 * 12 + 18) * r        # read U (two rows) and own staples, write G
BYTES_DIRECT = lambda r: (18 + 18) * r                   # read U, write G

# Fat-link path force (asqtad/HISQ smearing), flop per link of each kernel, counted from
# the kernel source: SU(3) product 198, product accumulated into a matrix 216, matrix
# axpy 36, matrix scaling or addition 18.
FAT_FLOP = {"fat_fk1": 2754, "fat_fk2": 7722, "fat_fk3": 2916, "fat_bk3": 2538, "fat_bk2": 8010,
            "fat_gk": 23418}
# minimum HBM matrices (18 reals) read + written per link by each kernel
FAT_MATRICES = {"fat_fk1": 4, "fat_fk2": 10, "fat_fk3": 9, "fat_bk3": 5, "fat_bk2": 12, "fat_gk": 22}
C_ASQTAD = (5 / 8, -1 / 16, 1 / 64, -1 / 384, -1 / 16, -1 / 24)

# Wilson-clover force, flop per link (force kernel: 6 clover plaquettes of 8 products
# each with the insertions, hopping outer products, U B' and C' U^+, TA) and per link of
# the clover-insertion pass (6 colour matrices per site from X, Y); minimum bytes per
# link in reals: force = U (two rows) + G + a quarter of the site's X, Y (24 complex) and
# K (six anti-Hermitian matrices, 9 reals each).
WILSON_FLOP = {"wilson_force": 11262, "wilson_clover": 500}
WILSON_REALS = {"wilson_force": 12 + 18 + (48 + 54) / 4, "wilson_clover": (48 + 54) / 4}
KAPPA, CSW = 0.1242, 1.37

PEAK = {"f32": 157.3e12, "f64": 78.6e12}   # MI355X vector peaks (FP32 counts packed FMA)
PEAK_F32_NONPACKED = 78.6e12               # 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_HBM = 8.0e12

TRAFFIC_FILES = {p: os.path.join(ROOT, "profiles", f"force_factored_{p}_32x32x32x64_traffic.json")
                 for p in ("f32", "f64")}
KERNEL_SOURCES = ["force_factored.hip", "factored.hpp", "su3.hpp", "lattice.hpp", "kernels.hpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1808_02281_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counters, or
    None when absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILES[prec]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_force(sym, torch, U, L, u0, beta, steps, warmup):
    """Time `steps` force calls with the fused action (no profiling hooks in the timed
    loop), then the same number again with per-kernel HIP events for the kernel split."""
    F = torch.empty_like(U)
    for _ in range(warmup):
        sym.force(U, L, u0, beta, with_action=True, out=F)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    S = None
    for _ in range(steps):
        _, S = sym.force(U, L, u0, beta, with_action=True, out=F)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / steps
    sym.profile_enable(True)
    sym.profile_collect()
    for _ in range(steps):
        sym.force(U, L, u0, beta, with_action=True, out=F)
    torch.cuda.synchronize()
    kernels = sym.profile_collect()
    sym.profile_enable(False)
    return ms, wall, kernels, F, S.cpu().numpy()


def force_error_report(G, G_ref, S, S_ref):
    """Errors of a GPU force and action against the oracle's, in the norms the tests
    gate: max over links of the Frobenius error / max over links of the reference norm,
    the RMS ratio, the worst per-link relative error and where it is, and |S - S_ref|/|S_ref|."""
    import numpy as np

    d = np.sqrt(np.sum(np.abs(G - G_ref) ** 2, axis=(-2, -1))).reshape(-1)
    r = np.sqrt(np.sum(np.abs(G_ref) ** 2, axis=(-2, -1))).reshape(-1)
    rel = d / np.maximum(r, 1e-300)
    k = int(np.argmax(rel))
    return {"force_max_rel": float(d.max() / r.max()),
            "force_rms_rel": float(np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(r * r))),
            "force_worst_link_rel": float(rel[k]),
            "worst_link": {"site": k // 4, "mu": k % 4},
            "action_rel": float(abs(S - S_ref) / abs(S_ref))}


def bench_batch(sym, torch, gaugegen, u0, beta, reps=20):
    """64 independent lattices of uneven sizes (8^4, 12^4, 16^3x32; eps in [0.2, 0.4]),
    FP32 force with FP64 action: per-lattice calls against one batched launch per pass,
    eager and replayed from a captured HIP graph."""
    recipe = gaugegen.batch_recipe(64, 6)
    dev = torch.device("cuda:0")
    Ls = [r["L"] for r in recipe]
    Us = []
    for i, r in enumerate(recipe):
        Us.append(sym.pack(gaugegen.near_thermal_links_device(r["L"], r["eps"], r["seed"], dev, torch.complex64),
                           r["L"]))
        if i % 16 == 15:
            torch.cuda.synchronize()
            log(f"  generated {i + 1} of {len(recipe)} lattices")
    links = sum(4 * sym.volume(L) for L in Ls)
    Fs = [torch.empty_like(U) for U in Us]
    S = torch.empty((len(Us), 4), dtype=torch.float64, device=dev)

    def per_lattice():
        for U, L, F in zip(Us, Ls, Fs):
            sym.force(U, L, u0, beta, with_action=True, out=F)

    def batched():
        sym.force_batch(Us, Ls, u0, beta, with_action=True, out=Fs, S_out=S)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def graphed(fn):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return timed(g.replay)

    out = {"lattices": len(Us), "links": links, "sizes": {"8^4": Ls.count((8, 8, 8, 8)),
                                                          "12^4": Ls.count((12, 12, 12, 12)),
                                                          "16^3x32": Ls.count((16, 16, 16, 32))}}
    ms = timed(per_lattice)
    out["per_lattice_eager"] = {"ms": ms, "link_forces_per_s": links / (ms * 1e-3), "launches": 3 * len(Us)}
    ms = graphed(per_lattice)
    out["per_lattice_graph"] = {"ms": ms, "link_forces_per_s": links / (ms * 1e-3)}
    ms = timed(batched)
    out["batched_default"] = {"ms": ms, "link_forces_per_s": links / (ms * 1e-3), "launches": 3}
    best, tune_log = sym.batch_autotune(Us, Ls, u0, beta)
    ms = timed(batched)
    out["batched_tuned"] = {"ms": ms, "link_forces_per_s": links / (ms * 1e-3), "schedule": best}
    out["autotune_log"] = [{**c, "ms": t} for c, t in tune_log]
    ms = graphed(batched)
    out["batched_tuned_graph"] = {"ms": ms, "link_forces_per_s": links / (ms * 1e-3)}
    return out


def bench_fat(sym, torch, U_np, L, steps, warmup, with_fp64=True, with_cpu=True, budget_s=8.0):
    """Fat-link path force on the same lattice: synthetic adjoint fields GV, GW (complex
    Gaussian per matrix element, seed 7, standing in for the fermion outer products),
    asqtad coefficients; one step = sym_fat_force in gradient mode (5 kernels)."""
    import numpy as np

    dev = torch.device("cuda:0")
    V = int(np.prod(L))
    links = 4 * V
    rng = np.random.default_rng(7)
    shape = U_np.shape
    GV_np = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    GW_np = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    out = {"workload": f"{WORKLOAD}, adjoint fields complex Gaussian (seed 7), asqtad coefficients",
           "coefficients": list(C_ASQTAD)}
    for prec, cdt in (("f32", torch.complex64), ("f64", torch.complex128)):
        if prec == "f64" and not with_fp64:
            continue
        U = sym.pack(torch.from_numpy(U_np).to(dev).to(cdt), L)
        GV = sym.pack(torch.from_numpy(GV_np).to(dev).to(cdt), L)
        GW = sym.pack(torch.from_numpy(GW_np).to(dev).to(cdt), L)
        g = torch.empty_like(U)
        for _ in range(warmup):
            sym.fat_force(U, L, C_ASQTAD, GV, GW, mode="grad", out=g)
        torch.cuda.synchronize()
        sym.profile_enable(True)
        sym.profile_collect()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            sym.fat_force(U, L, C_ASQTAD, GV, GW, mode="grad", out=g)
        e1.record()
        torch.cuda.synchronize()
        kern = sym.profile_collect()
        ms = e0.elapsed_time(e1) / steps
        # forward smearing (fat and Naik links)
        Vf, Wf = torch.empty_like(U), torch.empty_like(U)
        sym.fat_links(U, L, C_ASQTAD, out=(Vf, Wf))
        torch.cuda.synchronize()
        sym.profile_collect()
        e0.record()
        for _ in range(steps):
            sym.fat_links(U, L, C_ASQTAD, out=(Vf, Wf))
        e1.record()
        torch.cuda.synchronize()
        kern_f = sym.profile_collect()
        sym.profile_enable(False)
        ms_f = e0.elapsed_time(e1) / steps
        # the HMC pattern: fat links, then the force reusing their intermediates
        wsr = sym.new_fat_workspace(L, sym.prec_of(U.dtype), U.device)
        sym.fat_links(U, L, C_ASQTAD, out=(Vf, Wf), ws=wsr)
        sym.fat_force(U, L, C_ASQTAD, GV, GW, mode="grad", out=g, ws=wsr, reuse_links=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            sym.fat_links(U, L, C_ASQTAD, out=(Vf, Wf), ws=wsr)
            sym.fat_force(U, L, C_ASQTAD, GV, GW, mode="grad", out=g, ws=wsr, reuse_links=True)
        e1.record()
        torch.cuda.synchronize()
        ms_lf = e0.elapsed_time(e1) / steps
        del wsr
        r = 4 if prec == "f32" else 8
        per = {}
        for name, (tot, n) in list(kern.items()) + [(k, v) for k, v in kern_f.items() if k == "fat_fk3"]:
            t = tot / n * 1e-3
            per[name] = {"ms": t * 1e3, "tflops": FAT_FLOP[name] * links / t / 1e12,
                         "min_hbm_tbs": FAT_MATRICES[name] * 18 * r * links / t / 1e12}
        gk = per["fat_gk"]
        peak = PEAK[prec]
        res = {"value": links / (ms * 1e-3), "unit": "link-forces/s", "ms_per_step": ms,
               "fat_links_ms": ms_f, "links_then_force_reusing_ms": ms_lf, "kernels": per,
               "roofline": {"kernel": "fat_gk", "bound": "alu", "achieved": gk["tflops"], "peak": peak / 1e12,
                            "unit": "TFLOP/s", "frac": gk["tflops"] * 1e12 / peak,
                            "flop_per_link": FAT_FLOP["fat_gk"],
                            "hbm_min_bytes_per_link": FAT_MATRICES["fat_gk"] * 18 * r,
                            "hbm_frac_at_min_bytes": gk["min_hbm_tbs"] * 1e12 / PEAK_HBM}}
        out[prec] = res
        log(f"  fat path force {prec}: {ms:.3f} ms/step, fat links {ms_f:.3f} ms, links then force reusing "
            f"their intermediates {ms_lf:.3f} ms; {per}")
        del U, GV, GW, g, Vf, Wf
    if with_cpu:
        import oracle

        n = 64
        while True:
            sites = rng.integers(0, V, n)
            mus = rng.integers(0, 4, n).astype(np.int32)
            t0 = time.perf_counter()
            oracle.fat_grad_links(U_np, L, C_ASQTAD, GV_np, GW_np, sites, mus)
            dt = time.perf_counter() - t0
            if dt >= budget_s / 4:
                break
            n = int(n * max(2.0, budget_s / max(dt, 1e-3) * 0.9))
        out["cpu_oracle"] = {"value": n / dt, "unit": "link-forces/s", "cores": oracle.num_threads(),
                             "kind": "oracle", "sample": f"{n} random links, FP64 per-path algorithm ({dt:.1f} s)"}
    return out


def bench_wilson(sym, torch, U_np, L, steps, warmup, with_fp64=True, with_cpu=True, budget_s=6.0):
    """Wilson-clover fermion force on the same lattice for synthetic X, Y (complex Gaussian
    spinors, seeds 8 and 9; kappa 0.1242, c_sw 1.37); one step = sym_wilson_force."""
    import numpy as np

    dev = torch.device("cuda:0")
    V = int(np.prod(L))
    links = 4 * V
    rng = np.random.default_rng(8)
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    X_np = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    rng = np.random.default_rng(9)
    Y_np = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    out = {"workload": f"{WORKLOAD}, X and Y complex Gaussian spinors (seeds 8, 9)", "kappa": KAPPA, "csw": CSW}
    for prec, cdt in (("f32", torch.complex64), ("f64", torch.complex128)):
        if prec == "f64" and not with_fp64:
            continue
        U = sym.pack(torch.from_numpy(U_np).to(dev).to(cdt), L)
        X = sym.pack_spinor(torch.from_numpy(X_np).to(dev).to(cdt), L)
        Y = sym.pack_spinor(torch.from_numpy(Y_np).to(dev).to(cdt), L)
        G = torch.empty_like(U)
        for _ in range(warmup):
            sym.wilson_force(U, X, Y, L, KAPPA, CSW, out=G)
        torch.cuda.synchronize()
        sym.profile_enable(True)
        sym.profile_collect()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            sym.wilson_force(U, X, Y, L, KAPPA, CSW, out=G)
        e1.record()
        torch.cuda.synchronize()
        kern = sym.profile_collect()
        sym.profile_enable(False)
        ms = e0.elapsed_time(e1) / steps
        r = 4 if prec == "f32" else 8
        per = {}
        for name, (tot, n) in kern.items():
            t = tot / n * 1e-3
            per[name] = {"ms": t * 1e3, "tflops": WILSON_FLOP[name] * links / t / 1e12,
                         "min_hbm_tbs": WILSON_REALS[name] * r * links / t / 1e12}
        fk = per["wilson_force"]
        peak = PEAK[prec]
        out[prec] = {"value": links / (ms * 1e-3), "unit": "link-forces/s", "ms_per_step": ms, "kernels": per,
                     "roofline": {"kernel": "wilson_force", "bound": "alu", "achieved": fk["tflops"],
                                  "peak": peak / 1e12, "unit": "TFLOP/s", "frac": fk["tflops"] * 1e12 / peak,
                                  "flop_per_link": WILSON_FLOP["wilson_force"],
                                  "hbm_min_bytes_per_link": WILSON_REALS["wilson_force"] * r,
                                  "hbm_frac_at_min_bytes": fk["min_hbm_tbs"] * 1e12 / PEAK_HBM}}
        log(f"  wilson force {prec}: {ms:.3f} ms/step; {per}")
        del U, X, Y, G
    if with_cpu:
        import oracle

        n = 256
        while True:
            sites = rng.integers(0, V, n)
            mus = rng.integers(0, 4, n).astype(np.int32)
            t0 = time.perf_counter()
            oracle.wilson_force_links(U_np, X_np, Y_np, L, KAPPA, CSW, sites, mus)
            dt = time.perf_counter() - t0
            if dt >= budget_s / 4:
                break
            n = int(n * max(2.0, budget_s / max(dt, 1e-3) * 0.9))
        out["cpu_oracle"] = {"value": n / dt, "unit": "link-forces/s", "cores": oracle.num_threads(),
                             "kind": "oracle", "sample": f"{n} random links, FP64 ({dt:.1f} s)"}
    return out


def bench_autograd(sym, torch, gaugegen, u0, beta, steps, warmup):
    """Differentiation on the 24^3x48 workload (links eps 0.3, seed 3): S_G through
    torch autograd, forward = force kernels with the fused action (2 G U per link kept
    for the backward), backward = scaling by the incoming gradient; one step = forward
    + backward."""
    cfg = gaugegen.CONFIGS["thermal_24x24x24x48"]
    L = cfg["L"]
    dev = torch.device("cuda:0")
    links = 4 * sym.volume(L)
    aos = gaugegen.near_thermal_links_device(L, cfg["eps"], cfg["seed"], dev)
    out = {"workload": "thermal_24x24x24x48", "links": links}
    for prec, cdt in (("f32", torch.complex64), ("f64", torch.complex128)):
        U = sym.pack(aos.to(cdt), L).requires_grad_(True)

        def step():
            U.grad = None
            S = sym.symanzik_action(U, L, u0, beta)
            S.backward()

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[prec] = {"ms_per_forward_backward": ms, "link_gradients_per_s": links / (ms * 1e-3)}
        log(f"  autograd {prec}: {ms:.3f} ms per forward + backward")
        del U
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(U_np, L, u0, beta, one_thread_budget_s=8.0):
    """The FP64 oracle's force on every link of the workload with OpenMP on all host
    threads (the timed value; its forces and action are kept for the error report), and
    on a random sample of links at one thread (the oracle's per-link gather, since the
    whole-field scatter at one thread would take minutes)."""
    import numpy as np

    import oracle

    c, _ = oracle.coeffs(u0)
    V = int(np.prod(L))
    threads = oracle.set_num_threads(os.cpu_count() or 1)
    t0 = time.perf_counter()
    G_ref = oracle.force(U_np, L, c, beta)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    S_ref = oracle.action(U_np, L, c, beta)[0]
    dt_action = time.perf_counter() - t1
    log(f"  oracle force on all {4 * V} links: {dt:.1f} s on {threads} threads; action {dt_action:.1f} s")
    one = oracle.set_num_threads(1)
    rng = np.random.default_rng(99)
    n = 2048
    while True:
        sites = rng.integers(0, V, n)
        mus = rng.integers(0, 4, n).astype(np.int32)
        t2 = time.perf_counter()
        oracle.force_links(U_np, L, c, beta, sites, mus)
        dt1 = time.perf_counter() - t2
        if dt1 >= one_thread_budget_s / 4:
            break
        n = int(n * max(2.0, one_thread_budget_s / max(dt1, 1e-3) * 0.9))
    oracle.set_num_threads(threads)
    base = {
        "value": 4 * V / dt,
        "unit": "link-forces/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"every link ({4 * V}) of the 32^3x64 workload, FP64, C oracle with OpenMP: every loop "
                  f"instance walked once, its staples scattered to its links ({dt:.1f} s)",
        "value_1_thread": n / dt1,
        "sample_1_thread": f"{n} random links of the same workload, one thread, each link's staples "
                           f"gathered by the force algorithm's rotation rules ({dt1:.1f} s)",
        "host_threads": os.cpu_count(),
        "cpu_model": cpu_model(),
    }
    return base, G_ref, S_ref


def copy_calibration(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def fma_rate(torch, dtype, iters=8192, reps=5):
    """Measured vector FMA throughput in TFLOP/s: the probe kernel of libsymprobe.so (a
    benchmark helper built beside libsym.so, not part of its ABI), best of ``reps``."""
    import ctypes

    path = os.path.join(ROOT, "paper_1808_02281_amd", "libsymprobe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP libraries first (__graft_entry__.build())")
    lib = ctypes.CDLL(path)
    lib.probe_fma.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.probe_fma.restype = ctypes.c_int
    prec = {torch.float32: 1, torch.float64: 2}[dtype]
    dev = torch.device("cuda:0")
    out = torch.empty(4096 * 256, dtype=dtype, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

    def call():
        rc = lib.probe_fma(prec, int(iters), ctypes.c_void_p(out.data_ptr()), stream)
        if rc != 0:
            raise RuntimeError(f"probe_fma failed with status {rc}")

    call()
    torch.cuda.synchronize(dev)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    if not torch.isfinite(out).all():
        raise RuntimeError("FMA probe produced non-finite values")
    return 2.0 * 8 * iters * 4096 * 256 / (best * 1e-3) / 1e12


def measured_peaks(sym, torch):
    """Device rates the roofline fractions can be read against: vector FMA throughput
    (the probe kernel: non-packed FP32 and FP64 FMAs, as the library's kernels are compiled) and HBM bandwidth of a
    plain 2 GiB device copy (read + write) and fill (write), best of 5."""
    res = {"fp32_fma_tflops": fma_rate(torch, torch.float32), "fp64_fma_tflops": fma_rate(torch, torch.float64)}
    n = 1 << 29  # 2 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            t = ms if t is None else min(t, ms)
        return t * 1e-3

    res["hbm_copy_tbs"] = 2 * 4 * n / best(lambda: b.copy_(a)) / 1e12
    res["hbm_write_tbs"] = 4 * n / best(lambda: b.fill_(2.0)) / 1e12
    del a, b
    log(f"  measured peaks: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-md", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fat", action="store_true", help="skip the fat-link path force")
    ap.add_argument("--no-wilson", action="store_true", help="skip the Wilson-clover force")
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd timing")
    ap.add_argument("--only-f32", action="store_true", help="profiling runs: FP32 force only")
    ap.add_argument("--only-f64", action="store_true", help="profiling runs: FP64 force only")
    ap.add_argument("--only-force", action="store_true", help="profiling runs: FP32 and FP64 force only")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the device peak measurements")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the force would shard by domain decomposition along t, exchanging two t-slices of links "
              "per side).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return

    import gaugegen
    import paper_1808_02281_amd as sym

    if args.only_f32 or args.only_f64 or args.only_force:
        args.no_cpu_baseline = args.no_md = args.no_batch = args.no_fat = True
        args.no_wilson = args.no_autograd = args.no_peaks = True
        args.no_fp64 = args.only_f32

    cfg = gaugegen.CONFIGS[WORKLOAD]
    L = cfg["L"]
    u0, beta = gaugegen.U0, gaugegen.BETA
    V = int(np.prod(L))
    links = 4 * V
    dev = torch.device("cuda:0")

    log(f"generating {WORKLOAD} (eps={cfg['eps']}, seed={cfg['seed']})")
    t0 = time.perf_counter()
    U_np = gaugegen.near_thermal_links(L, cfg["eps"], cfg["seed"])
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    aos = torch.from_numpy(U_np).to(dev)
    U32 = sym.pack(aos.to(torch.complex64), L)
    U64 = None if args.no_fp64 else sym.pack(aos, L)
    del aos
    torch.cuda.synchronize()

    log("timing FP32 force")
    ms32, wall32, k32, F32, S32 = time_force(sym, torch, U32, L, u0, beta, args.steps, args.warmup)
    value = links / (ms32 * 1e-3)
    log(f"  {ms32:.3f} ms/step, kernels {k32}")

    def kernel_avg(kernels, name):
        tot, n = kernels.get(name, (0.0, 0))
        return tot / n if n else None

    def roofline_of(kernels, prec):
        dom = "force_factored" if "force_factored" in kernels else "force_direct"
        t_dom = kernel_avg(kernels, dom) * 1e-3
        flop_dom = FLOP_FACTORED if dom == "force_factored" else FLOP_DIRECT
        bytes_dom = (BYTES_FACTORED if dom == "force_factored" else BYTES_DIRECT)(4 if prec == "f32" else 8)
        alu = flop_dom * links / t_dom
        hbm = bytes_dom * links / t_dom
        r = {
            "kernel": dom,
            "bound": "alu",
            "achieved": alu / 1e12,
            "peak": PEAK[prec] / 1e12,
            "unit": "TFLOP/s",
            "frac": alu / PEAK[prec],
            "traffic": measured_traffic(prec) if dom == "force_factored" else None,
            "flop_per_link": flop_dom,
            "hbm_min_bytes_per_link": bytes_dom,
            "hbm_frac_at_min_bytes": hbm / PEAK_HBM,
            "kernel_ms": t_dom * 1e3,
        }
        if prec == "f32":
            r["frac_of_nonpacked_fp32_peak"] = alu / PEAK_F32_NONPACKED
        if r["traffic"]:
            # FETCH_SIZE/WRITE_SIZE count bytes leaving the L2s, Infinity Cache hits included
            r["l2_egress_frac_of_hbm_peak"] = r["traffic"] / t_dom / PEAK_HBM
        return dom, r

    dom, roofline = roofline_of(k32, "f32")
    paper_equiv = FLOP_PAPER * value
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "link-forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "lattice": list(L), "links": links, "eps": cfg["eps"], "seed": cfg["seed"],
                   "u0": u0, "beta": beta, "precision": "f32 link products, f64 action reduction",
                   "algorithm": "factored" if dom == "force_factored" else "direct"},
        "roofline": roofline,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in k32.items()},
        "paper_equivalent": {"flop_per_link": FLOP_PAPER, "tflops": paper_equiv / 1e12,
                             "frac_of_fp32_peak": paper_equiv / PEAK["f32"]},
        "action_f32": S32.tolist(),
        "wall_s": wall32,
    }
    # the forces leave the GPU for the comparison with the oracle at the end
    G32_host = sym.unpack(F32, L).cpu().numpy() if not args.no_cpu_baseline else None
    G64_host = None
    del F32

    if not args.no_fp64:
        log("timing FP64 force")
        ms64, _, k64, F64, S64 = time_force(sym, torch, U64, L, u0, beta, args.steps, args.warmup)
        out["fp64"] = {"value": links / (ms64 * 1e-3), "ms_per_step": ms64,
                       "kernels_ms_per_step": {k: v[0] / args.steps for k, v in k64.items()},
                       "roofline": roofline_of(k64, "f64")[1],
                       "action": S64.tolist()}
        out["fp32_speedup_over_fp64"] = ms64 / ms32
        if not args.no_cpu_baseline:
            G64_host = sym.unpack(F64, L).cpu().numpy()
        del F64
        log(f"  {ms64:.3f} ms/step")

    if not args.no_md:
        log("timing FP32 leapfrog")
        P = sym.pack(torch.from_numpy(gaugegen.momenta(L, 4)).to(torch.complex64).to(dev), L)
        Um = U32.clone()
        nst = 4
        sym.md_leapfrog(Um, P, L, u0, beta, 0.02, 1, with_energy=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sym.md_leapfrog(Um, P, L, u0, beta, 0.02, nst, with_energy=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out["md_leapfrog"] = {"prec": "f32", "nsteps": nst, "dt": 0.02, "ms_per_step": ms / nst,
                              "link_updates_per_s": links * nst / (ms * 1e-3)}
        del P, Um

    if not args.no_autograd:
        log("timing autograd (24^3x48)")
        out["autograd"] = bench_autograd(sym, torch, gaugegen, u0, beta, args.steps, args.warmup)

    if not args.no_batch:
        log("timing the 64-lattice batch")
        out["batch"] = bench_batch(sym, torch, gaugegen, u0, beta)

    if not args.no_fat:
        log("timing the fat-link path force")
        del U32
        if U64 is not None:
            del U64
        torch.cuda.empty_cache()
        out["fat_path_force"] = bench_fat(sym, torch, U_np, L, args.steps, args.warmup, with_fp64=not args.no_fp64,
                                          with_cpu=not args.no_cpu_baseline)

    if not args.no_wilson:
        log("timing the Wilson-clover force")
        out["wilson_clover_force"] = bench_wilson(sym, torch, U_np, L, args.steps, args.warmup,
                                                  with_fp64=not args.no_fp64, with_cpu=not args.no_cpu_baseline)

    if not args.no_peaks:
        log("measuring device peaks")
        out["measured_peaks"] = measured_peaks(sym, torch)
        mp = out["measured_peaks"]["fp32_fma_tflops"]
        out["roofline"]["measured_peak"] = mp
        out["roofline"]["frac_of_measured_peak"] = out["roofline"]["achieved"] / mp
        if "fp64" in out:
            mp64 = out["measured_peaks"]["fp64_fma_tflops"]
            out["fp64"]["roofline"]["measured_peak"] = mp64
            out["fp64"]["roofline"]["frac_of_measured_peak"] = out["fp64"]["roofline"]["achieved"] / mp64

    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"], G_ref, S_ref = cpu_baseline(U_np, L, u0, beta)
        # errors of the timed results against the FP64 oracle on the same (unrounded)
        # links: end to end for FP32, whose kernel error on the rounded links is gated
        # at 1e-5 by the tests
        log("comparing with the oracle")
        err = {"reference": "FP64 oracle, every link of the workload, unrounded FP64 links",
               "f32": force_error_report(G32_host.astype(np.complex128), G_ref, S32[0], S_ref)}
        if G64_host is not None:
            err["f64"] = force_error_report(G64_host, G_ref, S64[0], S_ref)
        err["tolerance"] = {"f32": 1e-5, "f64": 1e-12}
        out["error_vs_oracle"] = err
        log(f"  {err}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
