"""Benchmark of the CPM apply and solve on one MI355X.

Workload: the torus R = 1, rho = 0.4 at h = 1/512 with two interior
Dirichlet circles (meridians at toroidal angles 0 and pi, second order), the
largest single-GPU configuration of the target set (34.1M PDE DOFs + 139k BC
DOFs; its vectors and stored closest points exceed the 256 MB Infinity
Cache, so HBM traffic is not hidden).

Timed step: one FP64 application of A = m I + n [diag L + (L - diag L) E]
(m = 0, n = -1: Poisson) to a vector resident in HBM; value = DOFs / step
time in Gnodes/s.  Also reported on the same line: the FP32 apply rate, the
per-phase time of the apply from HIP events on its stream, the roofline of
the dominant kernel (the tile gather) and of the whole apply, the transposed
apply, the time to a relative residual of 1e-8 for the mixed-precision and
the plain FP64 solve (median of repeated runs), the solves of the other
target configurations with their error against the oracle's solution
(stored by tests/golden/make_config_golden.py) and against the closed form,
the differentiable solve (forward, and backward through the adjoint solve),
the batched uneven solves (32 spheres and tori, h = 1/64 .. 1/192, 3
right-hand sides each) against one FP64 solve per instance, the paper's heat
test (Crank-Nicolson, sphere h = 1/256) with its error, the band build time,
and the FP64 CPU oracle timed on the host (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve]
       [--no-cpu] [--no-batch] [--no-adjoint] [--no-configs] [--N 512]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
BYTES_PER_ROW_F64 = 40.0   # per row of the apply: cp_S 24 + u 8 + v 8 (FP64)
BYTES_PER_ROW_F32 = 24.0   # fraction 12 + base 4 + u 4 + v 4 (FP32 vectors)
GOLDEN = os.path.join(ROOT, "tests", "golden")

# HBM bytes per launch of the FP64 tile gather on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; summaries and commands in
# profiles/gather_torus512_pmc.md), each scaled by the same counter's reading
# for a plain device copy of known size.  They hold only for the kernel
# source they were taken on: `traffic` is null when its hash differs.
GATHER_PMC = {"sources_sha1": "a2076ed167a9048b0227a02209f59ad9e8eeff7e",
              "fetch_bytes": 1.56062e+09, "write_bytes": 2.96609e+08}
# The same runs for the whole FP64 apply (tile gather, explicit E rows,
# Laplacian pass, explicit L rows; profiles/*_torus512_pmc.md), valid while
# the hash of apply.hip, lagrange.hpp and builder.hip is the one below.
APPLY_PMC = {"sources_sha1": "7d585bba18b378b84b2c81d24b10de2c2fb1a1e0",
             "bytes": {"tile gather": 1.85723e+09, "explicit E rows": 2.07567e+08,
                       "block Laplacian": 1.05252e+09, "explicit L rows": 1.61315e+07}}


def _code(text):
    """Source text with comments removed and whitespace collapsed, so that a
    change to comments or layout keeps the counters that were taken on the
    code."""
    import re
    text = re.sub(r'"(?:\\.|[^"\\\n])*"|//[^\n]*|/\*.*?\*/',
                  lambda m: m.group(0) if m.group(0).startswith('"') else " ", text, flags=re.S)
    return " ".join(text.split())


def gather_sources_sha1():
    """Hash of what sets the FP64 tile gather's traffic: its own source (the
    k_gather templates, the row and cube helpers they call, the Lagrange
    weights) and the band builder, which fixes the block order and tiles."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2305_04711_amd/csrc/apply.hip")).read()
    a = src.index("struct TileView {")
    b = src.index("template <class T>\n__device__ __forceinline__ T wave_sum")
    h = hashlib.sha1(_code(src[a:b]).encode())
    for f in ("lagrange.hpp", "builder.hip"):
        h.update(_code(open(os.path.join(ROOT, "paper_2305_04711_amd/csrc", f)).read()).encode())
    return h.hexdigest()


def apply_sources_sha1():
    """Hash of every source that sets the whole apply's traffic."""
    import hashlib
    h = hashlib.sha1()
    for f in ("apply.hip", "lagrange.hpp", "builder.hip"):
        h.update(_code(open(os.path.join(ROOT, "paper_2305_04711_amd/csrc", f)).read()).encode())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def median(xs):
    s = sorted(xs)
    k = len(s)
    return s[k // 2] if k % 2 else 0.5 * (s[k // 2 - 1] + s[k // 2])


def host_cpu():
    """(CPU model name, host threads this process may use; the box's share
    of the host is capped at 16)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, max(1, min(16, n or 1))


# --------------------------------------------------------------- CPU oracle
def cpu_baseline(threads):
    """The oracle as it stands (explicit CSR E and L, the four-step product of
    Sec. 5.4, numpy/scipy) on the host: its apply on the bench's torus and
    meridians at h = 1/128, one thread and `threads` threads at once on
    independent vectors (scipy's sparse products release the GIL), and its
    BiCGSTAB solve of the gauged sphere Poisson problem at h = 1/64 to 1e-8."""
    import threading
    import numpy as np
    from oracle import geometry as G
    from oracle import krylov as KR
    from oracle import operator as O
    from paper_2305_04711_amd import inputs
    t_all = time.perf_counter()
    T = G.Torus(1.0, 0.4)
    t0 = time.perf_counter()
    sysm = O.CPMSystem(T, 128, [G.MeridianC(T, 1.0, 0.0), G.MeridianC(T, -1.0, 0.0)])
    build_s = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    us = [rng.standard_normal(sysm.n) for _ in range(threads)]
    sysm.apply(us[0], 0.0, -1.0)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        sysm.apply(us[0], 0.0, -1.0)
    t1 = (time.perf_counter() - t0) / reps

    def work(u):
        for _ in range(reps):
            sysm.apply(u, 0.0, -1.0)

    th = [threading.Thread(target=work, args=(u,)) for u in us]
    t0 = time.perf_counter()
    for x in th:
        x.start()
    for x in th:
        x.join()
    tp = time.perf_counter() - t0
    n128 = sysm.n
    del sysm, us
    # the solve: C2 at h = 1/64 (gauged sphere Poisson), single thread
    S = G.Sphere()
    s2 = O.CPMSystem(S, 64, [])
    f = inputs.sphere_field(inputs.sphere_coeffs(1), s2.CP)
    b = s2.rhs(f, None, -1.0)
    mv = KR.gauge_matvec(lambda u: s2.apply(u, 0.0, -1.0), s2.n_s, 64.0 * 64.0)
    t0 = time.perf_counter()
    _, info = KR.bicgstab(mv, b, tol=1e-8)
    solve_s = time.perf_counter() - t0
    model, _ = host_cpu()
    out = {"value": threads * reps * n128 / tp / 1e9, "unit": "Gnodes/s", "cores": threads,
           "kind": "oracle",
           "sample": "FP64 oracle apply (explicit CSR E, L; four-step product; numpy/scipy) on "
                     "the bench's torus and meridian IBCs at h = 1/128 (%d DOFs): %d threads "
                     "running %d applies each on independent vectors in %.2f s; single "
                     "thread %.3f s per apply" % (n128, threads, reps, tp, t1),
           "cpu_model": model,
           "single_thread_gnodes_per_s": n128 / t1 / 1e9,
           "oracle_dofs": n128, "oracle_build_s": build_s,
           "solve_c2_h64": {"dofs": s2.n, "tol": 1e-8, "seconds": solve_s,
                            "iters": info["iters"], "relres": float(info["relres"]),
                            "threads": 1},
           "seconds_total": time.perf_counter() - t_all}
    log("cpu baseline: %s" % out)
    return out


# --------------------------------------------------------------- helpers
class DofIndex:
    """Grid coordinates (and curve, for BC DOFs) -> DOF of a GPU band."""

    def __init__(self, band):
        import numpy as np
        self.np = np
        K = band.coords().astype(np.int64)
        self.key = self._key(K)
        self.order = np.argsort(self.key)
        self.sk = self.key[self.order]
        self.n_s = band.n_s
        self.bc = {}
        if band.n_c:
            node, curve = band.bc_node(), band.bc_curve()
            for c in np.unique(curve):
                sel = np.nonzero(curve == c)[0]
                idx = np.full(band.n_s, -1, dtype=np.int64)
                idx[node[sel]] = band.n_s + sel
                self.bc[int(c)] = idx

    def _key(self, K):
        K = K.astype(self.np.int64) + (1 << 20)
        z = K[:, 2] if K.shape[1] == 3 else 0
        return (K[:, 0] << 42) | (K[:, 1] << 21) | z

    def pde(self, K):
        np = self.np
        k = self._key(np.asarray(K))
        p = np.minimum(np.searchsorted(self.sk, k), self.sk.size - 1)
        return np.where(self.sk[p] == k, self.order[p], -1)

    def bcdof(self, K, curve):
        d = self.pde(K)
        out = self.np.full(d.size, -1, dtype=self.np.int64)
        for c in self.np.unique(curve):
            m = curve == c
            out[m] = self.bc[int(c)][d[m]]
        return out


def vs_golden(band, x, name):
    """Relative L-infinity difference between a GPU solution and the oracle's
    stored solution at the golden file's DOFs."""
    import numpy as np
    g = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    assert int(g["n_s"]) == band.n_s and int(g["n_c"]) == band.n_c, name
    ix = DofIndex(band)
    d = ix.pde(g["pde_coords"])
    assert np.all(d >= 0)
    xs = x.cpu().numpy()
    got, ref = [xs[d]], [g["pde_u"]]
    if "bc_coords" in g.files:
        db = ix.bcdof(g["bc_coords"], g["bc_curve"])
        assert np.all(db >= 0)
        got.append(xs[db])
        ref.append(g["bc_u"])
    got, ref = np.concatenate(got), np.concatenate(ref)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))), int(ref.size), float(g["relres"])


def inner_nodes(band, depth_h=2.0):
    """PDE DOFs within depth_h grid spacings of the surface, where the
    solution is the closest-point extension of the surface values up to the
    discretisation error (nodes further out only serve the FD stencils)."""
    import numpy as np
    X = band.coords() / float(band.N)
    cp = band.cp()
    d = np.sqrt(((X - cp) ** 2).sum(1))
    return np.nonzero(d <= depth_h / band.N)[0], cp


def timed_solve(band, b, m, n, tol, mode, reps, **kw):
    import torch
    from paper_2305_04711_amd import cpm
    secs, x, st = [], None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, st = cpm.solve(band, b, m, n, tol=tol, mode=mode, raise_noconv=False, **kw)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t)
    return x, st, secs


def solve_record(st, secs):
    return {"seconds": median(secs), "runs_s": secs, "converged": bool(st["converged"]),
            "relres": st["relres"], "krylov_iters": st["krylov_iters"],
            "outer_iters": st["outer_iters"], "restarts": st["restarts"],
            "fallback_f64": bool(st["fallback_f64"])}


# --------------------------------------------------------------- configs
def run_configs(dev):
    """C1, C2, C3 of the target set: each solve's error against the oracle's
    solution (golden files) and against the closed form."""
    import numpy as np
    import torch
    from paper_2305_04711_amd import cpm, inputs
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from closed_forms import circle_point_dirichlet, latitude_harmonic, sphere_poisson
    out = {}
    # C1: unit circle h = 1/32, point Dirichlet u(1, 0) = 0, GMRES(50) to 1e-10
    band = cpm.Band(cpm.circle(), [cpm.point_ibc((1.0, 0.0), (0.0, 1.0))], 32)
    cp = band.cp()
    f, (a, bb) = inputs.circle_source(0, cp)
    b = cpm.rhs(band, torch.tensor(f, device=dev),
                torch.zeros(band.n_c, dtype=torch.float64, device=dev), -1.0)
    x, st, secs = timed_solve(band, b, 0.0, -1.0, 1e-10, "gmres", 5, restart=50)
    err, cnt, orr = vs_golden(band, x, "solve_c1_circle32.npz")
    inner, cpi = inner_nodes(band)
    th = np.arctan2(cpi[inner, 1], cpi[inner, 0])
    ca = 0.1 * a.copy()
    ca[2] += 1.0
    ex = circle_point_dirichlet(th, 0.0, ca, 0.1 * bb)
    cf = float(np.max(np.abs(x.cpu().numpy()[inner] - ex)))
    out["c1_circle_h32_gmres"] = dict(solve_record(st, secs), dofs=band.n, tol=1e-10,
                                      rel_linf_vs_oracle=err, oracle_dofs_compared=cnt,
                                      oracle_relres=orr, linf_vs_closed_form=cf)
    log("C1: %s" % out["c1_circle_h32_gmres"])
    # C2: unit sphere h = 1/64, gauged Poisson with seeded harmonics l <= 8
    band = cpm.Band(cpm.sphere(), [], 64)
    co = inputs.sphere_coeffs(1)
    cpt = torch.tensor(band.cp(), device=dev)
    b = cpm.rhs(band, inputs.sphere_field(co, cpt), None, -1.0)
    inner, cpi = inner_nodes(band)
    ex = sphere_poisson(co, cpi[inner])
    res = {"dofs": band.n}
    for mode in ("f64", "mixed"):
        for tol, reps in ((1e-8, 5), (1e-12, 1)):
            x, st, secs = timed_solve(band, b, 0.0, -1.0, tol, mode, reps, gauge=64.0 * 64.0)
            err, cnt, orr = vs_golden(band, x, "solve_c2_sphere64.npz")
            u = x.cpu().numpy()[inner]
            cf = float(np.max(np.abs((u - u.mean()) - (ex - ex.mean()))))
            res["%s_tol%.0e" % (mode, tol)] = dict(solve_record(st, secs), tol=tol,
                                                    rel_linf_vs_oracle=err,
                                                    linf_vs_closed_form=cf)
    res["oracle_dofs_compared"], res["oracle_relres"] = cnt, orr
    res["speedup_mixed_tol1e-8"] = res["f64_tol1e-08"]["seconds"] / res["mixed_tol1e-08"]["seconds"]
    out["c2_sphere_h64"] = res
    log("C2: %s" % res)
    # C3: unit sphere, latitude z = 0.3 with u = sin 2 phi, f = 0; h = 1/64
    # against the oracle, h = 1/256 (the configuration's size) mixed vs FP64
    for N in (64, 256):
        band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], N)
        cpc = band.bc_cpc()
        g = torch.tensor(np.sin(2.0 * np.arctan2(cpc[:, 1], cpc[:, 0])), device=dev)
        b = cpm.rhs(band, torch.zeros(band.n_s, dtype=torch.float64, device=dev), g, -1.0)
        inner, cpi = inner_nodes(band)
        ex = latitude_harmonic(cpi[inner], 0.3)
        res = {"dofs": band.n, "n_c": band.n_c}
        xs = {}
        plan = ((1e-8, 5), (1e-12, 1)) if N == 64 else ((1e-8, 3),)
        for mode in ("f64", "mixed"):
            for tol, reps in plan:
                x, st, secs = timed_solve(band, b, 0.0, -1.0, tol, mode, reps)
                rec = dict(solve_record(st, secs), tol=tol,
                           linf_vs_closed_form=float(np.max(np.abs(x.cpu().numpy()[inner] - ex))))
                if N == 64:
                    err, cnt, orr = vs_golden(band, x, "solve_c3_latitude64.npz")
                    rec["rel_linf_vs_oracle"] = err
                    res["oracle_dofs_compared"], res["oracle_relres"] = cnt, orr
                res["%s_tol%.0e" % (mode, tol)] = rec
                xs[(mode, tol)] = x
        res["speedup_mixed_tol1e-8"] = res["f64_tol1e-08"]["seconds"] / res["mixed_tol1e-08"]["seconds"]
        a64, a32 = xs[("f64", 1e-8)], xs[("mixed", 1e-8)]
        res["mixed_vs_f64_rel_linf_tol1e-8"] = ((a32 - a64).abs().max() / a64.abs().max()).item()
        out["c3_latitude_h%d" % N] = res
        log("C3 h=1/%d: %s" % (N, res))
        del xs
    return out


def run_batch(dev, args):
    """Batched uneven solves: 32 instances (even k: unit sphere, odd k: torus
    R = 1, rho = 0.4) at N_k = 64 + round(128 k / 31), 3 right-hand sides
    each (seeded smooth sources), screened Poisson (m = 1, n = -1), to a
    relative residual of 1e-8: batched mixed precision and batched FP64
    against the plain FP64 solve of each instance one call at a time."""
    import torch
    from paper_2305_04711_amd import cpm, inputs
    bands, t0 = [], time.perf_counter()
    for k in range(32):
        N = 64 + int(round(128 * k / 31))
        if k % 2 == 0:
            bands.append(cpm.Band(cpm.sphere(), [], N))
        else:
            bands.append(cpm.Band(cpm.torus(1.0, 0.4), [], N))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    nrhs = 3
    batch = cpm.Batch(bands, [1.0] * 32, [-1.0] * 32, nrhs=nrhs)
    tune = batch.autotune(torch.float32)
    tune64 = batch.autotune(torch.float64)
    b = torch.empty(nrhs, batch.total, dtype=torch.float64, device=dev)
    for k, band in enumerate(bands):
        cp = torch.tensor(band.cp(), device=dev)
        lo, hi = batch.offsets[k], batch.offsets[k + 1]
        for r in range(nrhs):
            if k % 2 == 0:
                fv = inputs.sphere_field(inputs.sphere_coeffs(100 + k + 1000 * r, lmin=0), cp)
            else:
                fv = inputs.torus_field(inputs.torus_coeffs(100 + k + 1000 * r), cp)
            b[r, lo:hi] = fv
    out = {"instances": 32, "nrhs": nrhs, "dofs_total": batch.total,
           "dofs_min": min(bd.n for bd in bands), "dofs_max": max(bd.n for bd in bands),
           "build_s": build_s, "autotune_f32": tune, "autotune_f64": tune64}
    xs = {}
    for mode in ("mixed", "f64"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, st = batch.solve(b, tol=1e-8, mode=mode, raise_noconv=False)
        torch.cuda.synchronize()
        xs[mode] = x
        out["batched_" + mode] = {
            "seconds": time.perf_counter() - t,
            "converged": all(s["converged"] for s in st),
            "max_relres": max(s["relres"] for s in st),
            "max_krylov_iters": max(s["krylov_iters"] for s in st),
            "fallback_f64_systems": sum(s["fallback_f64"] for s in st)}
        log("batched %s: %s" % (mode, out["batched_" + mode]))
    # plain FP64 solves, one instance (3 right-hand sides) per call
    torch.cuda.synchronize()
    t = time.perf_counter()
    worst, conv, diff = 0.0, True, 0.0
    for k, band in enumerate(bands):
        lo, hi = batch.offsets[k], batch.offsets[k + 1]
        xk, st = cpm.solve(band, b[:, lo:hi].contiguous(), 1.0, -1.0, tol=1e-8, mode="f64",
                           raise_noconv=False)
        worst = max(worst, st["relres"])
        conv = conv and bool(st["converged"])
        for mode in ("mixed", "f64"):
            xb = xs[mode][:, lo:hi]
            diff = max(diff, ((xb - xk).abs().max() / xk.abs().max()).item())
    torch.cuda.synchronize()
    out["sequential_f64"] = {"seconds": time.perf_counter() - t, "converged": conv,
                             "max_relres": worst}
    out["batched_vs_sequential_rel_linf"] = diff
    out["speedup_vs_sequential_f64"] = {
        mode: out["sequential_f64"]["seconds"] / out["batched_" + mode]["seconds"]
        for mode in ("mixed", "f64")}
    log("sequential f64: %s" % out["sequential_f64"])
    del batch, bands, xs
    return out


def run_variant(dev, args, N, m, n, dt64_cubic, solves_cubic, n_tube, **kw):
    """The same torus and interior boundaries with another discretisation
    choice (quadratic interpolation, p = 2, Sec. 7; or the stencil-set band,
    Sec. 5.1): band size, FP64 apply time and the FP64 solve to 1e-8, beside
    the cubic tube's figures."""
    import torch
    from paper_2305_04711_amd import cpm, inputs
    t0 = time.perf_counter()
    band = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                          cpm.meridian_ibc(-1.0, 0.0)], N, order=2, **kw)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    cpm.autotune(band, torch.float64, 1, reps=10)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    u = torch.randn(band.n, device=dev, dtype=torch.float64, generator=gen)
    for _ in range(args.warmup):
        v = cpm.apply(band, u, m, n)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        v = cpm.apply(band, u, m, n)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    del v
    out = {"dofs": band.n, "n_s": band.n_s, "n_c": band.n_c, "dofs_vs_tube": band.n / n_tube,
           "build_s": build_s, "apply_f64_ms": dt * 1e3, "gnodes_per_s": band.n / dt / 1e9,
           "apply_speedup_vs_cubic_tube": dt64_cubic / dt}
    if solves_cubic is not None:
        cp = band.cp()
        f = torch.tensor(inputs.torus_field(inputs.torus_coeffs(100), cp), device=dev)
        g = torch.tensor(inputs.meridian_dirichlet(band.bc_cpc(), seed=2), device=dev)
        b = cpm.rhs(band, f, g, n)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, st = cpm.solve(band, b, m, n, tol=1e-8, mode="f64", raise_noconv=False)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        out["solve_f64"] = {"seconds": sec, "converged": bool(st["converged"]),
                            "relres": st["relres"], "krylov_iters": st["krylov_iters"],
                            "speedup_vs_cubic_tube": solves_cubic["f64"]["seconds"] / sec}
    log("variant %s: %s" % (kw, out))
    return out


def run_heat(dev, N=256):
    """The heat test of Sec. 6.2 at h = 1/N: unit sphere, exact solution
    exp(-2t) z, second-order Dirichlet IBC on the circle z = 0.3 with the exact
    solution as data, Crank-Nicolson with dt = 0.1 h to t = 0.1 (N steps),
    FP64 solves to 1e-10 warm-started from the previous step."""
    import numpy as np
    import torch
    from paper_2305_04711_amd import cpm
    band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], N, order=2)
    cp = band.cp()
    dt = 0.1 / N
    nsteps = N
    u0 = np.empty(band.n)
    u0[:band.n_s] = cp[:, 2]
    u0[band.n_s:] = u0[band.bc_node()]
    zc = band.bc_cpc()[:, 2]
    g = np.exp(-2.0 * dt * np.arange(nsteps + 1))[:, None] * zc[None, :]
    u0t = torch.tensor(u0, device=dev)
    gt = torch.tensor(g, device=dev)
    cpm.heat_cn(band, u0t, dt, 2, gt[:3].contiguous(), tol=1e-10)     # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    u, st = cpm.heat_cn(band, u0t, dt, nsteps, gt, tol=1e-10)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    X = band.coords() / float(N)
    depth = np.abs(np.sqrt((X * X).sum(1)) - 1.0)
    keep = (depth <= np.sqrt(17.0) / N - 1.0 / N) & (np.abs(cp[:, 2] - 0.3) > 0.2)
    err = np.max(np.abs(u.cpu().numpy()[:band.n_s][keep] - np.exp(-0.2) * cp[keep, 2]))
    out = {"N": N, "dofs": band.n, "steps": nsteps, "seconds": sec,
           "ms_per_step": sec / nsteps * 1e3, "krylov_iters": st["krylov_iters"],
           "converged": bool(st["converged"]), "linf_err_vs_exact": err}
    log("heat: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--solve-reps", type=int, default=3,
                    help="runs per mode of the time-to-1e-8 solve (the median is reported)")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation run")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the C1 / C2 / C3 solves against the oracle's solutions")
    ap.add_argument("--no-quadratic", action="store_true",
                    help="skip the quadratic-interpolation (p = 2) and stencil-set bands")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (a kernel of known "
                         "traffic for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the band would shard by surface patch, with halo exchanges per apply)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_04711_amd import cpm, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    N = args.N
    m, n = 0.0, -1.0

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    band = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                          cpm.meridian_ibc(-1.0, 0.0)], N, order=2)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = band.info
    log("band: n_s %d n_c %d blocks %d tiles %d built in %.3f s" %
        (band.n_s, band.n_c, info["n_blocks"], info["n_tiles"], build_s))

    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    u64 = torch.randn(band.n, device=dev, dtype=torch.float64, generator=gen)
    u32 = u64.float()
    v64 = torch.empty_like(u64)
    v32 = torch.empty_like(u32)
    lib, h = band._lib, band.handle
    import ctypes as C

    def apply_once(u, v, code):
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        r = lib.cpm_apply(h, m, n, code, 1, C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()), st)
        if r != 0:
            raise RuntimeError(lib.cpm_last_error().decode())

    def timed(u, v, code):
        for _ in range(args.warmup):
            apply_once(u, v, code)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            apply_once(u, v, code)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.steps

    tune64 = cpm.autotune(band, torch.float64, 1, reps=10)
    tune32 = cpm.autotune(band, torch.float32, 1, reps=10)
    log("autotune f64 %s, f32 %s" % (tune64, tune32))
    dt64 = timed(u64, v64, 0)
    dt32 = timed(u32, v32, 1)
    ph64, _ = cpm.apply_profile(band, u64, m, n, reps=max(10, args.steps))
    ph32, _ = cpm.apply_profile(band, u32, m, n, reps=max(10, args.steps))
    # rows processed by the tile gather = PDE rows without swapped members
    tile_rows = band.n_s - (info["n_erows"] - band.n_c)
    ach64 = BYTES_PER_ROW_F64 * tile_rows / (ph64[0] * 1e-3) / 1e9
    ach32 = BYTES_PER_ROW_F32 * tile_rows / (ph32[0] * 1e-3) / 1e9
    log("apply f64 %.4f ms (%.2f Gnodes/s), phases %s" % (dt64 * 1e3, band.n / dt64 / 1e9, ph64))
    log("apply f32 %.4f ms (%.2f Gnodes/s), phases %s" % (dt32 * 1e3, band.n / dt32 / 1e9, ph32))

    def transpose_once(u, v, code):
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        r = lib.cpm_apply_transpose(h, m, n, code, 1, C.c_void_p(u.data_ptr()),
                                    C.c_void_p(v.data_ptr()), st)
        if r != 0:
            raise RuntimeError(lib.cpm_last_error().decode())

    def timed_T(u, v, code, reps=10):
        for _ in range(2):
            transpose_once(u, v, code)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            transpose_once(u, v, code)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    dtT64 = timed_T(u64, v64, 0)
    dtT32 = timed_T(u32, v32, 1)
    log("transpose apply f64 %.4f ms, f32 %.4f ms" % (dtT64 * 1e3, dtT32 * 1e3))
    traffic = None
    if GATHER_PMC["sources_sha1"] is not None and GATHER_PMC["sources_sha1"] == gather_sources_sha1():
        traffic = GATHER_PMC["fetch_bytes"] + GATHER_PMC["write_bytes"]
    apply_traffic = None
    if APPLY_PMC["sources_sha1"] == apply_sources_sha1():
        apply_traffic = sum(APPLY_PMC["bytes"].values())
    del u32, v32

    solves = None
    if not args.no_solve:
        cp = band.cp()
        f = torch.tensor(inputs.torus_field(inputs.torus_coeffs(100), cp), device=dev)
        g = torch.tensor(inputs.meridian_dirichlet(band.bc_cpc(), seed=2), device=dev)
        b = cpm.rhs(band, f, g, n)
        solves = {}
        xs = {}
        for mode in ("mixed", "f64"):
            x, st, secs = timed_solve(band, b, m, n, 1e-8, mode, args.solve_reps)
            xs[mode] = x
            solves[mode] = solve_record(st, secs)
            log("solve %s: %s" % (mode, solves[mode]))
        # both solutions meet the same residual; their difference reflects
        # the conditioning of A at this h (about kappa * 1e-8), not a
        # precision loss
        solves["mixed_vs_f64_rel_linf"] = ((xs["mixed"] - xs["f64"]).abs().max()
                                           / xs["f64"].abs().max()).item()
        solves["speedup_mixed"] = solves["f64"]["seconds"] / solves["mixed"]["seconds"]
        del xs

    adjoint = None
    if not args.no_solve and not args.no_adjoint:
        # forward + backward of the differentiable solve (loss against a seeded
        # smooth target): one adjoint solve plus the RHS adjoint
        t_np = inputs.torus_field(inputs.torus_coeffs(3), cp)
        tt = torch.tensor(t_np, device=dev)
        fr = f.clone().requires_grad_(True)
        gr = g.clone().requires_grad_(True)
        stats = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        # FP64 BiCGSTAB: the FP32 recurrence needs more iterations than it
        # saves per iteration (forward and transposed operator alike)
        u = cpm.CPMSolve.apply(fr, gr, band, m, n, 1e-8, "f64", stats)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t
        loss = ((u[:band.n_s] - tt) ** 2).sum()
        t = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        adjoint = {"forward_s": t_fwd, "backward_s": time.perf_counter() - t,
                   "tol": 1e-8, "mode": "f64", "grad_f_norm": fr.grad.norm().item(),
                   "grad_g_norm": gr.grad.norm().item(),
                   "forward_iters": stats["forward"]["krylov_iters"],
                   "backward_iters": stats["backward"]["krylov_iters"],
                   "backward_fallback_f64": bool(stats["backward"]["fallback_f64"])}
        log("adjoint: %s" % adjoint)

    quad = ssb = None
    if not args.no_quadratic:
        quad = run_variant(dev, args, N, m, n, dt64, solves, band.n, p=2)
        ssb = run_variant(dev, args, N, m, n, dt64, solves, band.n, band="stencil_set")

    # the apply at the oracle's size of this workload (h = 1/128), for the
    # GPU / CPU ratio at equal size
    small = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                           cpm.meridian_ibc(-1.0, 0.0)], 128, order=2)
    cpm.autotune(small, torch.float64, 1, reps=10)
    us = torch.randn(small.n, device=dev, dtype=torch.float64, generator=gen)
    for _ in range(args.warmup):
        cpm.apply(small, us, m, n)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        cpm.apply(small, us, m, n)
    torch.cuda.synchronize()
    dt_small = (time.perf_counter() - t) / args.steps
    apply_h128 = {"dofs": small.n, "ms": dt_small * 1e3, "gnodes_per_s": small.n / dt_small / 1e9}
    del small, us

    del band, u64, v64
    if solves is not None:
        del b, f, g
    torch.cuda.empty_cache()

    configs = None
    if not args.no_configs:
        configs = run_configs(dev)

    batch_out = None
    if not args.no_batch:
        batch_out = run_batch(dev, args)

    heat_out = None
    if not args.no_solve and not args.no_heat:
        heat_out = run_heat(dev)

    # a plain 1 GiB device copy (1 GiB read + 1 GiB written per copy): the
    # bandwidth a streaming kernel reaches on this device, beside the 8 TB/s
    # peak; with --calibrate-copy the counter runs also see its dispatches
    src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3 if args.calibrate_copy else 1):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / 10
    copy_gbs = 2.0 * src.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del src, dst
    log("1 GiB device copy: %.3f ms, %.0f GB/s" % (copy_ms, copy_gbs))
    model, threads = host_cpu()
    base = None if args.no_cpu else cpu_baseline(threads)
    dofs = info["n"]
    gn64, gn32 = dofs / dt64 / 1e9, dofs / dt32 / 1e9
    out = {
        "metric": "Gnodes/s of CPM apply (% HBM peak) + time-to-1e-8 solve, mixed vs FP64",
        "value": gn64,
        "unit": "Gnodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "torus R=1 rho=0.4, h=1/%d, two second-order Dirichlet meridian "
                               "IBCs (toroidal angles 0, pi); Poisson m=0 n=-1" % N,
                   "n_s": info["n_s"], "n_c": info["n_c"], "dofs": dofs},
        "roofline": {"bound": "hbm", "kernel": "k_gather<double,3,1> (tile gather a = E u)",
                     "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach64 / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_row": BYTES_PER_ROW_F64, "rows_per_launch": tile_rows,
                     "launch_ms": ph64[0]},
        "apply_roofline": {"f64": {"gnodes_per_s": gn64, "bytes_per_row": BYTES_PER_ROW_F64,
                                   "achieved_gbs": gn64 * BYTES_PER_ROW_F64,
                                   "frac": gn64 * BYTES_PER_ROW_F64 / HBM_PEAK_GBS,
                                   "traffic": apply_traffic,
                                   "traffic_vs_algorithmic": None if apply_traffic is None else
                                   apply_traffic / (BYTES_PER_ROW_F64 * dofs)},
                           "f32": {"gnodes_per_s": gn32, "bytes_per_row": BYTES_PER_ROW_F32,
                                   "achieved_gbs": gn32 * BYTES_PER_ROW_F32,
                                   "frac": gn32 * BYTES_PER_ROW_F32 / HBM_PEAK_GBS}},
        "copy_ceiling": {"gbs": copy_gbs, "ms": copy_ms, "bytes_per_copy": 2 * 2 ** 30,
                         "gather_frac_of_copy": ach64 / copy_gbs},
        "cpu_baseline": base,
        "gpu_vs_cpu_at_h128": None if base is None else {
            "gpu_apply_gnodes_per_s": apply_h128["gnodes_per_s"],
            "cpu_apply_gnodes_per_s": base["value"], "cpu_threads": base["cores"],
            "ratio": apply_h128["gnodes_per_s"] / base["value"]},
        "apply_h128": apply_h128,
        "apply_f32": {"gnodes_per_s": gn32, "ms": dt32 * 1e3,
                      "gather_gbs": ach32, "gather_frac": ach32 / HBM_PEAK_GBS},
        "transpose_apply_ms": {"f64": dtT64 * 1e3, "f32": dtT32 * 1e3},
        "apply_phase_ms": {"f64": ph64, "f32": ph32,
                           "order": ["tile gather", "explicit E rows", "block Laplacian",
                                     "explicit L rows"]},
        "time_to_1e-8": solves,
        "configs": configs,
        "autotune": {"variants": "k = 8 * lap + 2 * mode + pad (mode 0 block order, 1 XCD-aware, 2 persistent XCD-aware gather, 3 persistent pipelined gather; lap 0..3 the forms of the Laplacian pass, 3 = two blocks per wave with scalar metadata)", "f64_ms": tune64[0], "f64_best": tune64[1],
                     "f32_ms": tune32[0], "f32_best": tune32[1]},
        "build_band_s": build_s,
        "adjoint": adjoint,
        "batched": batch_out,
        "heat_cn": heat_out,
        "quadratic_p2": quad,
        "stencil_set_band": ssb,
        "host": {"cpu_model": model, "threads_available": threads,
                 "gpu": torch.cuda.get_device_name(0)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
