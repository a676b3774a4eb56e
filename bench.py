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
the dominant kernel (the tile gather), the transposed apply, the time to a
relative residual of 1e-8 for the mixed-precision and the plain FP64 solve,
the differentiable solve (forward, and backward through the adjoint solve),
the batched uneven solves (32 spheres and tori, h = 1/64 .. 1/192, 3
right-hand sides each) against one FP64 solve per instance, the paper's heat
test (Crank-Nicolson, sphere h = 1/256) with its error, the band build time,
and the FP64 CPU oracle timed on the host (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve]
       [--no-cpu] [--no-batch] [--no-adjoint] [--N 512]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
BYTES_PER_ROW_F64 = 40.0   # tile gather: cp_S 24 + u 8 + a 8 (FP64)
BYTES_PER_ROW_F32 = 24.0   # tile gather: fraction 12 + base 4 + u 4 + a 4 (FP32)

# HBM bytes per launch of the FP64 tile gather on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; summaries and commands in
# profiles/gather_torus512_pmc.md), each scaled by the same counter's reading
# for a plain device copy of known size.  They hold only for the kernel
# source they were taken on: `traffic` is null when its hash differs.
GATHER_PMC = {"sources_sha1": "b1c8cb90e7a9f14f5b26e931871ddf54e1f24d66",
              "fetch_bytes": 1.49399e+09, "write_bytes": 2.96511e+08}
def gather_sources_sha1():
    """Hash of what sets the FP64 tile gather's traffic: its own source (the
    k_gather templates, the row and cube helpers they call, the Lagrange
    weights) and the band builder, which fixes the block order and tiles."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2305_04711_amd/csrc/apply.hip")).read()
    a = src.index("struct TileView {")
    b = src.index("template <class T>\n__device__ __forceinline__ T wave_sum")
    h = hashlib.sha1(src[a:b].encode())
    for f in ("lagrange.hpp", "builder.hip"):
        h.update(open(os.path.join(ROOT, "paper_2305_04711_amd/csrc", f), "rb").read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(seconds=12.0):
    """The oracle as it stands (explicit CSR E and L, four-step product) on
    the same geometry and interior boundaries at N = 64."""
    import numpy as np
    from oracle import geometry as G
    from oracle import operator as O
    T = G.Torus(1.0, 0.4)
    sysm = O.CPMSystem(T, 64, [G.MeridianC(T, 1.0, 0.0), G.MeridianC(T, -1.0, 0.0)])
    u = np.random.default_rng(0).standard_normal(sysm.n)
    sysm.apply(u, 0.0, -1.0)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        sysm.apply(u, 0.0, -1.0)
        k += 1
    dt = (time.perf_counter() - t0) / k
    return {"value": sysm.n / dt / 1e9, "unit": "Gnodes/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 oracle apply (explicit CSR E, L; four-step product; numpy/scipy, "
                      "single thread) on the same torus with the same two meridian IBCs at "
                      "h = 1/64 (%d DOFs), %d applies over %.1f s" % (sysm.n, k, k * dt)}


def run_batch(dev, args):
    """Batched uneven solves: 32 instances (even k: unit sphere, odd k: torus
    R = 1, rho = 0.4) at N_k = 64 + round(128 k / 31), 3 right-hand sides
    each (seeded smooth sources), screened Poisson (m = 1, n = -1), to a
    relative residual of 1e-8: batched mixed precision and batched FP64
    against the plain FP64 solve of each instance one call at a time."""
    import numpy as np
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
    for mode in ("mixed", "f64"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, st = batch.solve(b, tol=1e-8, mode=mode, raise_noconv=False)
        torch.cuda.synchronize()
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
    worst, conv = 0.0, True
    for k, band in enumerate(bands):
        lo, hi = batch.offsets[k], batch.offsets[k + 1]
        xk, st = cpm.solve(band, b[:, lo:hi].contiguous(), 1.0, -1.0, tol=1e-8, mode="f64",
                           raise_noconv=False)
        worst = max(worst, st["relres"])
        conv = conv and bool(st["converged"])
    torch.cuda.synchronize()
    out["sequential_f64"] = {"seconds": time.perf_counter() - t, "converged": conv,
                             "max_relres": worst}
    out["speedup_vs_sequential_f64"] = {
        mode: out["sequential_f64"]["seconds"] / out["batched_" + mode]["seconds"]
        for mode in ("mixed", "f64")}
    log("sequential f64: %s" % out["sequential_f64"])
    del batch, bands
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
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation run")
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

    import numpy as np
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

    solves = None
    if not args.no_solve:
        cp = band.cp()
        f = torch.tensor(inputs.torus_field(inputs.torus_coeffs(100), cp), device=dev)
        g = torch.tensor(inputs.meridian_dirichlet(band.bc_cpc(), seed=2), device=dev)
        b = cpm.rhs(band, f, g, n)
        solves = {}
        xs = {}
        for mode in ("mixed", "f64"):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, st = cpm.solve(band, b, m, n, tol=1e-8, mode=mode, raise_noconv=False)
            torch.cuda.synchronize()
            xs[mode] = x
            solves[mode] = {"seconds": time.perf_counter() - t, "converged": bool(st["converged"]),
                            "relres": st["relres"], "krylov_iters": st["krylov_iters"],
                            "outer_iters": st["outer_iters"],
                            "fallback_f64": bool(st["fallback_f64"])}
            log("solve %s: %s" % (mode, solves[mode]))
        # both solutions meet the same residual; their difference reflects
        # the conditioning of A at this h, not a precision loss
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
        torch.cuda.synchronize()
        t = time.perf_counter()
        u = cpm.CPMSolve.apply(fr, gr, band, m, n, 1e-8, "mixed")
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t
        loss = ((u[:band.n_s] - tt) ** 2).sum()
        t = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        adjoint = {"forward_s": t_fwd, "backward_s": time.perf_counter() - t,
                   "tol": 1e-8, "grad_f_norm": fr.grad.norm().item(),
                   "grad_g_norm": gr.grad.norm().item()}
        log("adjoint: %s" % adjoint)

    quad = ssb = None
    if not args.no_quadratic:
        quad = run_variant(dev, args, N, m, n, dt64, solves, band.n, p=2)
        ssb = run_variant(dev, args, N, m, n, dt64, solves, band.n, band="stencil_set")

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
    base = None if args.no_cpu else cpu_baseline()
    out = {
        "metric": "Gnodes/s of CPM apply (% HBM peak) + time-to-1e-8 solve, mixed vs FP64",
        "value": band.n / dt64 / 1e9,
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
                   "n_s": band.n_s, "n_c": band.n_c, "dofs": band.n},
        "roofline": {"bound": "hbm", "kernel": "k_gather<double,3,1> (tile gather a = E u)",
                     "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach64 / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_row": BYTES_PER_ROW_F64, "rows_per_launch": tile_rows,
                     "launch_ms": ph64[0]},
        "copy_ceiling": {"gbs": copy_gbs, "ms": copy_ms, "bytes_per_copy": 2 * 2 ** 30,
                         "gather_frac_of_copy": ach64 / copy_gbs},
        "cpu_baseline": base,
        "apply_f32": {"gnodes_per_s": band.n / dt32 / 1e9, "ms": dt32 * 1e3,
                      "gather_gbs": ach32, "gather_frac": ach32 / HBM_PEAK_GBS},
        "transpose_apply_ms": {"f64": dtT64 * 1e3, "f32": dtT32 * 1e3},
        "apply_phase_ms": {"f64": ph64, "f32": ph32,
                           "order": ["tile gather", "explicit E rows", "block Laplacian",
                                     "explicit L rows"]},
        "time_to_1e-8": solves,
        "autotune": {"variants": "k = 2 * mode + pad (mode 0 block order, 1 XCD-aware, 2 persistent XCD-aware gather)", "f64_ms": tune64[0], "f64_best": tune64[1],
                     "f32_ms": tune32[0], "f32_best": tune32[1]},
        "build_band_s": build_s,
        "adjoint": adjoint,
        "batched": batch_out,
        "heat_cn": heat_out,
        "quadratic_p2": quad,
        "stencil_set_band": ssb,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
