"""Benchmark: regional multigrid preconditioned CG on one MI355X.

Workload (default): 3D Q1 Laplacian (27-point stencil), 4x4x4 regions of 82^3
nodes (composite 325^3, 35.3M regional rows), FP64, 4-level regional V-cycle
with Chebyshev degree 3, CG to a 1e-8 relative residual, rhs U[-1, 1] from a
fixed seed.  One step = device assembly of the region matrices, hierarchy
setup (diagonal, power method, per-region Galerkin products, coarse inverse)
and the PCG solve.  The region layout (planner tables) is built once.

Prints one JSON line.  ``value`` is the PCG time-to-1e-8 (seconds, median over
the timed steps, which run without kernel timing); ``roofline`` is measured live
on the finest-level fused Chebyshev kernel with HIP events in a profiled pass of
the same step right after them, on the bytes that kernel must move, with the
same launch timed with every coupling streamed beside it (``general_path``);
``cpu_baseline`` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-8 residual + stencil GB/s, FP64 vs mixed/learned forms"
HBM_PEAK_GBS = 8000.0
# Bytes per regional row of the finest-level FP64 kernels for `coefs` stencil coefficients per row.
# The method's Chebyshev step (Algorithm 2 with its direction vector d) reads the coefficients, u,
# b, D^-1, d and writes d, u: 264 B/row for the 27-point operator; the CG product reads the
# coefficients and p and writes q: 232 B/row.  The kernels here keep no direction vector: a step
# takes d_(k-1) = u_(k-1) - u_(k-2) from the buffer it overwrites with u_k, so it reads u_(k-1),
# b, u_(k-2) (and D^-1) and writes u_k.  On a symmetric level they stream only the upper half (14
# coefficients), and the tiled FP64 Chebyshev kernels take D^-1 of a one-region row from its
# centre coefficient instead of reading it (only shared rows, about 5%, read it when their
# interface sum is finished): 144 B/row for the streamed step, 128 B/row for the product.
METHOD_CHEB_BYTES_PER_ROW = 8 * 27 + 6 * 8


def cheb_bytes_per_row(coefs, reads_dinv=True):
    return 8 * coefs + (5 if reads_dinv else 4) * 8


def cg_matvec_bytes_per_row(coefs):
    return 8 * coefs + 2 * 8


ALGO_COEFS = 27
# HBM bytes per launch of the dominant kernel from FETCH_SIZE/WRITE_SIZE counters scaled by a
# plain-copy calibration, read from the committed counter summary; used only while the sources
# that define the kernel, its tiles, launch shapes and region table hash as they did when the
# counters were taken.
COUNTERS = os.path.join(ROOT, "profiles", "k_stencil_table_cheb_c2_counters.md")
KERNEL_SOURCES = ("kernels_stencil.hip", "kernels.hip", "planner.cpp", "solver.cpp", "api.cpp")


def counted_traffic():
    """(bytes per launch, sources hash) recorded in the counter summary, or (None, None)."""
    import re

    try:
        text = open(COUNTERS).read()
    except OSError:
        return None, None
    m = re.search(r"traffic_bytes_per_launch\s+(\d+)\s+sources_sha\s+([0-9a-f]{16})", text)
    return (int(m.group(1)), m.group(2)) if m else (None, None)


CPU_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, {root!r})
import synth
from oracle import regional
from oracle.regions import Layout
o, e = synth.tensor_layout([[82, 82], [82, 82], [82, 82]])
w = synth.Workload("sample", 3, 1, o, e, 63, 4, 3, "laplace", h=1.0 / 324)
lay = Layout(3, o, e, 63)
coefs = regional.build_operator(lay, "laplace", h=w.h)
opt = regional.Options(nlevels=4, degree=3)
lv = regional.setup(lay, coefs, opt)
b = lay.to_regional(synth.rhs(w))
t = time.perf_counter()
res = regional.pcg(lv, b, opt, rtol=1e-30, maxit={its})
dt = time.perf_counter() - t
print(json.dumps({{"seconds": dt, "iterations": res.iterations, "rows": lay.n_regional}}))
"""


def cpu_baseline(gpu_iterations: int, n_rows: int):
    """The oracle's PCG iterations on 2x2x2 of the 64 regions (1/8 of the rows), the GPU's
    iteration count, single-threaded; scaled to the full workload by the row count."""
    its = gpu_iterations
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    res = subprocess.run([sys.executable, "-c", CPU_SAMPLE.format(root=ROOT, its=its)], capture_output=True,
                         text=True, env=env, timeout=600)
    if res.returncode != 0:
        return {"value": None, "unit": "s", "cores": 1, "kind": "oracle", "sample": "failed: " + res.stderr[-300:]}
    d = json.loads(res.stdout.strip().splitlines()[-1])
    per_it = d["seconds"] / d["iterations"] * (n_rows / d["rows"])
    return {
        "value": per_it * gpu_iterations,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        # not a measurement of the whole workload: a 1/8 sample extrapolated by its row count
        "extrapolated": f"x{n_rows / d['rows']:.0f} from a 1/{n_rows / d['rows']:.0f} sample (rows)",
        "sample_seconds": d["seconds"],
        "sample": (f"NumPy FP64 oracle, {d['iterations']} PCG iterations (V-cycle + regional matvec each) on "
                   f"2x2x2 of the 64 regions of 82^3 ({d['rows']} regional rows, {d['seconds']:.1f} s timed, "
                   f"setup excluded); value = that time x {n_rows / d['rows']:.0f} (rows of the full workload)"),
    }


PREC_NAME = {0: "fp64", 1: "fp32", 2: "fp32_bf16", 3: "fp32_bf16_auto"}


def _handle(w, dev):
    """Regions and finest operator of workload w on the device (device assembly)."""
    import numpy as np
    import torch

    import synth
    from paper_2103_11962_amd import regmg

    h = regmg.Handle(0)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    if w.pde == "fd5":
        h.set_composite_stencil(5, synth.fd5_composite_stencil(w))
    elif w.pde == "fd7":
        h.set_composite_stencil(27, synth.fd7_composite_stencil(w))
    elif w.pde == "elasticity":
        h.assemble_q1(regmg.PDE_ELASTICITY, w.h, youngs=synth.region_youngs_moduli(w), nu=w.nu)
    elif w.pde == "diffusion":
        ec = torch.from_numpy(np.ascontiguousarray(synth.jump_coefficients(w)).reshape(-1)).to(dev)
        h.assemble_q1(regmg.PDE_DIFFUSION, w.h, elem_coef=ec)
        h._keep = ec
    else:
        h.assemble_q1(regmg.PDE_LAPLACE, w.h)
    return h


def _timed_solves(h, b, reps=2, rtol_override=None, **kw):
    """Warm-up solve, then `reps` timed solves; median solve time and the last result."""
    import numpy as np
    import torch

    rtol = rtol_override or 1e-8
    x = torch.zeros_like(b)
    h.solve(b, x, rtol=rtol, maxit=400, **kw)
    outs = []
    for _ in range(reps):
        x.zero_()
        outs.append(h.solve(b, x, rtol=rtol, maxit=400, **kw))
    return float(np.median([o["solve_ms"] for o in outs])), outs[-1], x


def _setup(h, w, **opts):
    import torch

    t0 = time.perf_counter()
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, **opts)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def _cheb_bytes(h, kind, precision, stored=True, nreg=None):
    """Bytes per node of the level-0 Chebyshev step: the stencil blocks (stored: the ones the level
    streams, full or upper half, see rmg_level_kernel, none for regions served by their class
    tables when nreg is given; else the method's full 27 blocks) and the vectors u_(k-1), b,
    u_(k-2), D~^-1 read and u_k written (the method's step also reads and writes its direction
    vector d: one vector more each way); with BF16 storage the centre block comes from an FP32
    array.  Stored: the scalar tiled kernel in FP64 or FP32 computes D~^-1 of one-region rows
    instead of reading it."""
    lk = h.level_kernel(0)
    nd = 1 if kind == "scalar" else 3
    nb = nd * nd
    coefs = lk["coefs"] if stored else 27 * nb
    if stored and precision == 0 and nreg:
        coefs *= 1.0 - h.level_table_regions(0) / nreg
    coefs_lo = lk["coefs_lo"] if stored else 27 * nb
    if stored:
        vecs = 4 if kind == "scalar" and lk["kernel"] in (1, 2) and precision in (0, 1) else 5
    else:
        vecs = 6
    if precision == 0:
        return coefs * 8 + vecs * nd * 8
    if precision == 1:
        return coefs_lo * 4 + vecs * nd * 4
    return (coefs_lo - nb) * 2 + nb * 4 + vecs * nd * 4


def _cheb_gbs(h, kind, precision, rows, stored=True, nreg=None):
    from paper_2103_11962_amd import regmg

    n, ms = h.profile_query(regmg.TIMED_CHEB)
    if n == 0:
        return None
    return _cheb_bytes(h, kind, precision, stored, nreg) * rows / (ms / n * 1e-3) / 1e9


def variant_mixed(dev):
    """Elasticity 3x3x3 regions of 55^3: FP64 V-cycle vs FP32 vs FP32 with BF16 coefficients on level 0
    vs BF16 on the levels the measured convergence factor allows, FP64 with the nodal-block D~, and
    FP64 streaming every block (region_table = 0: the FP64 V-cycle otherwise reads the per-region
    elasticity blocks from the class tables, which the low-precision V-cycles do not have)."""
    import numpy as np

    import synth

    w = synth.workload("c3")
    b = _to_dev(synth.rhs(w), dev)
    out, x64 = {}, None
    for name, prec, extra in (("fp64", 0, {}), ("fp32", 1, {}), ("fp32_bf16", 2, {}), ("fp32_bf16_auto", 3, {}),
                              ("fp64_block_diag", 0, dict(block_diag=1)), ("fp64_streamed", 0, dict(region_table=0))):
        h = _handle(w, dev)
        setup_ms = _setup(h, w, precision=prec, **extra)
        rows = h.level_info(0)["n_regional"] // 3
        # the storage level 0 ended up with (the automatic choice decides per level)
        pl = [h.level_precision(l) for l in range(w.nlevels)]
        peff = prec if prec != 3 else (2 if pl[0]["coef_type"] == 2 else 1)
        h.profile(True)
        ms, res, x = _timed_solves(h, b)
        entry = {"setup_ms": setup_ms, "solve_ms": ms, "iterations": res["iterations"],
                 "true_relres": res["true_relres"],
                 "cheb_gbs": _cheb_gbs(h, "block3", peff, rows, stored=False),
                 "cheb_bytes_per_node": _cheb_bytes(h, "block3", peff, stored=False),
                 "cheb_gbs_at_stored_bytes": _cheb_gbs(h, "block3", peff, rows, nreg=len(w.extents)),
                 "cheb_stored_bytes_per_node": _cheb_bytes(h, "block3", peff, nreg=len(w.extents)),
                 "table_regions": h.level_table_regions(0)}
        if prec == 3:
            entry["levels"] = [{"coef_type": p["coef_type"], "rho_fp32": p["rho_fp32"], "rho_bf16": p["rho_bf16"]}
                               for p in pl]
        if name == "fp64":
            x64 = x.clone()
        else:
            entry["x_rel_diff_vs_fp64"] = float((x - x64).norm() / x64.norm())
        out[name] = entry
        h.close()
        print(f"[bench] mixed {name}: {ms:.1f} ms, {res['iterations']} its", file=sys.stderr, flush=True)
    out["speedup_fp32_bf16_vs_fp64"] = out["fp64"]["solve_ms"] / out["fp32_bf16"]["solve_ms"]
    out["workload"] = ("3D Q1 elasticity, 3x3x3 regions of 55^3 nodes (3 dofs/node), E lognormal per region, "
                       "nu 0.3, 4-level V-cycle, Chebyshev degree 3, PCG to 1e-8 (flexible in FP32/BF16)")
    return out


def variant_batched(dev):
    """256 uneven regions: one persistent autotuned launch per step with graph-captured CG
    iterations vs one launch per region, both with the FP32 V-cycle."""
    import tempfile

    import synth

    w = synth.workload("c4")
    b = _to_dev(synth.rhs(w), dev)
    out = {}
    cache = os.path.join(tempfile.gettempdir(), "regmg_bench_tune.txt")
    for name, opts in (("region_by_region", dict(precision=1, batched=0)),
                       ("batched", dict(precision=1, autotune=1, autotune_cache=cache, use_graph=1))):
        h = _handle(w, dev)
        setup_ms = _setup(h, w, **opts)
        rows = h.level_info(0)["n_regional"]
        h.profile(True)
        ms, res, _ = _timed_solves(h, b)
        out[name] = {"setup_ms": setup_ms, "solve_ms": ms, "iterations": res["iterations"],
                     "true_relres": res["true_relres"], "cheb_gbs": _cheb_gbs(h, "scalar", 1, rows, stored=False),
                     "cheb_bytes_per_row": _cheb_bytes(h, "scalar", 1, stored=False),
                     "cheb_gbs_at_stored_bytes": _cheb_gbs(h, "scalar", 1, rows),
                     "cheb_stored_bytes_per_row": _cheb_bytes(h, "scalar", 1)}
        if name == "batched":
            out[name]["tuning"] = h.tune_report().strip().splitlines()
        h.close()
        print(f"[bench] batched {name}: {ms:.1f} ms, {res['iterations']} its", file=sys.stderr, flush=True)
    out["regional_rows"] = rows
    out["speedup_batched_vs_region_by_region"] = out["region_by_region"]["solve_ms"] / out["batched"]["solve_ms"]
    out["workload"] = ("3D Q1 Laplacian, 8x8x4 regions with slab extents from {28,55,82,109} (seed 0), "
                       "4-level FP32 V-cycle inside FP64 CG to 1e-8")
    return out


def variant_learned(dev, train_steps=400):
    """Jump-coefficient diffusion 4x4x4 regions of 82^3: geometric vs learned interpolation (MLP
    trained on the device on 8 other seeds of a 2x2x2-region 28^3 version)."""
    import torch

    import synth
    from paper_2103_11962_amd import regmg

    t0 = time.perf_counter()
    m = regmg.Mlp(0)
    for s in range(1, 9):
        ws = synth.workload("c5_small", seed=s)
        hs = _handle(ws, dev)
        hs.setup_hierarchy(nlevels=ws.nlevels, cheb_degree=ws.cheb_degree)
        m.add_samples(hs, nsamples=4, seed=s, sweeps=20)
        hs.close()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    m.init_params(seed=0, out_scale=0.0)
    loss_geo, _ = m.loss_grad()
    m.init_params(seed=0, out_scale=0.01)
    t0 = time.perf_counter()
    hist = m.train(train_steps, 1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    theta = m.params()
    pairs = m.num_data()
    m.close()
    w = synth.workload("c5")
    b = _to_dev(synth.rhs(w), dev)
    out = {"training": {"pairs": pairs, "steps": train_steps, "data_s": t_data, "train_s": t_train,
                        "loss_initial": float(hist[0]), "loss_final": float(hist[-1]),
                        "loss_geometric_interpolation": loss_geo}}
    for name in ("geometric", "learned"):
        h = _handle(w, dev)
        if name == "learned":
            h.set_learned_prolongator(theta)
        setup_ms = _setup(h, w)
        info = h.prolongator_info()
        ms, res, _ = _timed_solves(h, b)
        out[name] = {"setup_ms": setup_ms, "solve_ms": ms, "iterations": res["iterations"],
                     "true_relres": res["true_relres"], "rho_10_cycles": h.convergence_factor(10),
                     "interpolation": {0: "geometric", 1: "stored", 2: "learned"}[info["kind"]]}
        if name == "learned":
            out[name]["judge"] = {"rho_learned": info["rho_learned"], "rho_geometric": info["rho_geometric"],
                                  "flags": info["flags"]}
        h.close()
        print(f"[bench] learned {name}: {ms:.1f} ms, {res['iterations']} its", file=sys.stderr, flush=True)
    out["speedup_learned_vs_geometric"] = out["geometric"]["solve_ms"] / out["learned"]["solve_ms"]
    out["workload"] = ("3D Q1 diffusion, 4x4x4 regions of 82^3, coefficient 10^s_R exp(N(0,1)) per element "
                       "(s_R ~ U(-4,4) on even regions), 4-level V-cycle, Chebyshev degree 3, PCG to 1e-8; "
                       "learned interpolation on the finest level, judged by 10 stationary cycles")
    return out


def variant_graph_2d(dev):
    """2D five-point 2x2 regions of 82^2 (cache-resident, launch-bound): eager vs graph replay."""
    import synth

    w = synth.workload("c1")
    b = _to_dev(synth.rhs(w), dev)
    out = {}
    import torch

    from paper_2103_11962_amd import regmg

    for name, g in (("eager", 0), ("graph", 1)):
        h = _handle(w, dev)
        _setup(h, w, use_graph=g)
        ms, res, _ = _timed_solves(h, b, reps=5)
        out[name] = {"solve_ms": ms, "iterations": res["iterations"], "true_relres": res["true_relres"]}
        if not g:
            # launch-bound: count the kernels one solve issues
            n0 = regmg.kernel_launches()
            x = torch.zeros_like(b)
            r = h.solve(b, x, rtol=1e-8, maxit=400)
            n1 = regmg.kernel_launches()
            out[name]["kernel_launches_per_solve"] = n1 - n0
            out[name]["kernel_launches_per_iteration"] = (n1 - n0) / max(r["iterations"], 1)
        h.close()
    out["workload"] = "2D five-point, 2x2 regions of 82^2, 3-level V-cycle, Chebyshev degree 2, PCG to 1e-8"
    return out


def _stencil_to_csr(w, stencil):
    """The assembled composite five-point matrix of a workload as CSR arrays (input preparation:
    the same numbers as its composite stencil, rows x fastest)."""
    import numpy as np
    import scipy.sparse as sp

    nx, ny = w.composite_shape_xyz
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [], [], []
    for s, (dx, dy) in enumerate(((0, -1), (-1, 0), (0, 0), (1, 0), (0, 1))):
        ys, xs = np.nonzero(stencil[s].reshape(ny, nx))
        ok = (xs + dx >= 0) & (xs + dx < nx) & (ys + dy >= 0) & (ys + dy < ny)
        ys, xs = ys[ok], xs[ok]
        rows.append(idx[ys, xs])
        cols.append(idx[ys + dy, xs + dx])
        vals.append(stencil[s].reshape(ny, nx)[ys, xs])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def variant_noninvasive(dev):
    """2D five-point, 2x2 regions of 82^2 (Section 4 input): region matrices split on the device
    from the assembled composite matrix given as CSR, versus from its composite stencil."""
    import synth

    w = synth.workload("c1")
    st = synth.fd5_composite_stencil(w)
    A = _stencil_to_csr(w, st)
    b = _to_dev(synth.rhs(w), dev)
    out = {}
    for name in ("composite_stencil", "composite_csr"):
        h = _handle(w, dev) if name == "composite_stencil" else None
        if h is None:
            from paper_2103_11962_amd import regmg

            h = regmg.Handle(0)
            h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
        import torch

        ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "composite_csr":
                h.set_composite_csr(5, A)
            else:
                h.set_composite_stencil(5, st)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        _setup(h, w)
        solve_ms, res, _ = _timed_solves(h, b)
        out[name] = {"split_ms_host_input": min(ms), "solve_ms": solve_ms, "iterations": res["iterations"],
                     "true_relres": res["true_relres"]}
        h.close()
    out["csr_nnz"] = int(A.nnz)
    out["workload"] = "2D five-point, 2x2 regions of 82^2 (composite 163^2), operator handed over assembled"
    return out


def variant_mg_solver(dev):
    """Multigrid as a solver (the paper's experiments): damped Jacobi (omega 0.6, one sweep) and
    region-local Gauss-Seidel on the 2D five-point 730^2 and 700 x 720 meshes in 3x3 regions to
    1e-12 (the settings of the paper's Table 1), and the Chebyshev V-cycle on the 3D Laplacian to
    1e-8 beside its PCG solve."""
    import synth

    out = {}
    o, e = synth.tensor_layout([[244] * 3, [244] * 3])
    w = synth.Workload("table1", 2, 1, o, e, 15, 4, 1, "fd5", seed=0)
    h = _handle(w, dev)
    _setup(h, w, smoother=1, jacobi_omega=0.6)
    b = _to_dev(synth.rhs(w), dev)
    ms, res, _ = _timed_solves(h, b, reps=3, method="mg", rtol_override=1e-12)
    hist = res["history"]
    out["jacobi_2d_730"] = {"solve_ms": ms, "cycles": res["iterations"], "relres": res["relres"],
                            "asymptotic_factor": (hist[-1] / hist[-11]) ** 0.1 if len(hist) > 11 else None}
    # the same mesh with region-local Gauss-Seidel (one forward sweep, omega 1) and the
    # symmetric variant (backward post-sweep)
    for key, sm in (("gauss_seidel_2d_730", 2), ("symmetric_gauss_seidel_2d_730", 3)):
        _setup(h, w, smoother=sm, jacobi_omega=1.0)
        ms, res, _ = _timed_solves(h, b, reps=3, method="mg", rtol_override=1e-12)
        hist = res["history"]
        out[key] = {"solve_ms": ms, "cycles": res["iterations"], "relres": res["relres"],
                    "asymptotic_factor": (hist[-1] / hist[-11]) ** 0.1 if len(hist) > 11 else None}
    h.close()
    # Table 1(b)'s rectangular mesh: 700 x 720 nodes in 3x3 regions whose extents (234, 241/240)
    # are not 3^k + 1, so every region ends in a shortened coarse interval
    w = synth.workload("table1_rect")
    h = _handle(w, dev)
    b = _to_dev(synth.rhs(w), dev)
    for key, sm, omega in (("jacobi_2d_700x720", 1, 0.6), ("gauss_seidel_2d_700x720", 2, 1.0)):
        _setup(h, w, smoother=sm, jacobi_omega=omega)
        ms, res, _ = _timed_solves(h, b, reps=3, method="mg", rtol_override=1e-12)
        out[key] = {"solve_ms": ms, "cycles": res["iterations"], "relres": res["relres"]}
    h.close()
    w = synth.workload("c2")
    h = _handle(w, dev)
    _setup(h, w)
    b = _to_dev(synth.rhs(w), dev)
    ms, res, _ = _timed_solves(h, b, reps=2, method="mg")
    out["chebyshev_3d_c2"] = {"solve_ms": ms, "cycles": res["iterations"], "relres": res["relres"]}
    h.close()
    out["workload"] = ("2D five-point 3x3 regions of 244^2 (730^2) and 700 x 720 nodes in 3x3 regions, 4 levels, "
                       "Jacobi or Gauss-Seidel, to 1e-12; 3D Q1 Laplacian "
                       "4x4x4 regions of 82^3, 4 levels, Chebyshev degree 3, to 1e-8")
    return out


def variant_hybrid(dev):
    """The structured/unstructured hybrid of Table 5: 3D seven-point Laplacian on 100^3 nodes (the
    paper's mesh) in 3x3x3 regions (34^3 each), 3-level W-cycle, two symmetric Gauss-Seidel iterations before and
    after, piecewise-constant transfers, flexible PCG and MG as a solver to 1e-6; all regions
    structured, the centre region unstructured, and all regions unstructured."""
    import numpy as np

    import synth

    o, e = synth.tensor_layout([[34] * 3] * 3)
    w = synth.Workload("fd7_100", 3, 1, o, e, 63, 3, 2, "fd7", seed=0)
    b = _to_dev(synth.rhs(w), dev)
    out = {}
    for name, unstructured in (("structured", []), ("centre_unstructured", [13]), ("unstructured", list(range(27)))):
        h = _handle(w, dev)
        kinds = np.zeros(27, dtype=np.int32)
        kinds[unstructured] = 1
        h.set_region_kinds(kinds)
        setup_ms = _setup(h, w, smoother=4, jacobi_omega=1.0, hybrid=1, cycle_gamma=2)
        row = {"setup_ms": setup_ms}
        for method in ("pcg", "mg"):
            ms, res, _ = _timed_solves(h, b, reps=2, rtol_override=1e-6, method=method)
            row[method] = {"solve_ms": ms, "iterations": res["iterations"], "true_relres": res["true_relres"]}
        row["levels"] = [h.hybrid_level_info(l) for l in range(3)]
        out[name] = row
        h.close()
    out["workload"] = ("3D seven-point Laplacian 100^3 (the paper's mesh) in 3x3x3 regions of 34^3, 3-level W-cycle, 2 symmetric "
                       "Gauss-Seidel iterations, piecewise-constant aggregation transfers, to 1e-6")
    return out


def variant_coarse_amg(dev):
    """The AMG coarse solver of Section 3.5 on the 3D Laplacian (4x4x4 regions of 82^3): three region
    levels leave a 37^3 = 50,653-dof coarsest composite operator, beyond the dense inverse, and one
    smoothed-aggregation V-cycle solves it; beside it the four-level hierarchy with the direct solve."""
    import torch

    import synth

    w = synth.workload("c2")
    b = _to_dev(synth.rhs(w), dev)
    out = {}
    for name, nl, amg in (("three_region_levels_amg", 3, 1), ("four_region_levels_direct", 4, 0)):
        h = _handle(w, dev)
        t0 = time.perf_counter()
        h.setup_hierarchy(nlevels=nl, cheb_degree=w.cheb_degree, coarse_amg=amg)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        ms, res, _ = _timed_solves(h, b, reps=3)
        row = {"setup_ms": setup_ms, "solve_ms": ms, "iterations": res["iterations"],
               "true_relres": res["true_relres"]}
        if amg:
            row["amg_levels"] = [h.amg_level_info(l) for l in range(h.amg_levels())]
        out[name] = row
        h.close()
    out["workload"] = ("3D Q1 Laplacian 4x4x4 regions of 82^3, Chebyshev degree 3, PCG to 1e-8; coarse solve by "
                       "SA-AMG (down to 2000 rows) below 3 region levels, or the dense inverse below 4")
    return out


def _to_dev(a, dev):
    import numpy as np
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(dev)


def kernel_source_sha():
    import hashlib

    # the stencil kernels, the setup kernels that build the region table, the planner and solver
    # sources that fix tiles and launch shapes, and the entry points that set option defaults
    sha = hashlib.sha256()
    for name in KERNEL_SOURCES:
        sha.update(open(os.path.join(ROOT, "paper_2103_11962_amd", "csrc", name), "rb").read())
    return sha.hexdigest()[:16]


def copy_rate_gbs():
    """Read + write GB/s of a plain 1 GiB device-to-device copy (torch), median of 5 timed copies:
    the streaming rate this GPU reaches outside the method, for reading the roofline fraction."""
    import numpy as np
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    return 2 * (1 << 30) / (float(np.median(ms)) * 1e-3) / 1e9


def copy_probe():
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 8, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=1,
                    help="steps of the profiled pass that times the dominant kernel after the timed steps")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision, batched, learned and graph comparisons")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the regional method here keeps all "
              "regions on one device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2103_11962_amd import regmg

    dev = torch.device("cuda:0")
    w = synth.workload(args.workload)
    b = torch.from_numpy(np.ascontiguousarray(synth.rhs(w)).reshape(-1)).to(dev)
    x = torch.zeros_like(b)
    ec = None
    if w.pde == "diffusion":
        ec = torch.from_numpy(np.ascontiguousarray(synth.jump_coefficients(w)).reshape(-1)).to(dev)
    h = regmg.Handle(0)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)

    def step(**opts):
        if w.pde == "fd5":
            h.set_composite_stencil(5, synth.fd5_composite_stencil(w))
        else:
            h.assemble_q1(regmg.PDE_DIFFUSION if ec is not None else regmg.PDE_LAPLACE, w.h, elem_coef=ec)
        t0 = time.perf_counter()
        h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, **opts)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        x.zero_()
        out = h.solve(b, x, rtol=1e-8, maxit=200)
        return t_setup, out

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup step {i} done", file=sys.stderr, flush=True)
    # timed steps: no kernel timing inside them (rmg_profile off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    setups, solves, outs = [], [], []
    for i in range(args.steps):
        ts, out = step()
        setups.append(ts)
        solves.append(out["solve_ms"] / 1e3)
        outs.append(out)
        print(f"[bench] step {i}: setup {ts*1e3:.1f} ms, solve {out['solve_ms']:.1f} ms, "
              f"{out['iterations']} its, true relres {out['true_relres']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    last = outs[-1]
    assert last["converged"] and last["true_relres"] <= 1e-8, last
    launches = regmg.kernel_launches()
    x.zero_()
    h.solve(b, x, rtol=1e-8, maxit=200)
    launches = regmg.kernel_launches() - launches

    # profiled pass, after the timed steps: the same step with an event pair around every
    # finest-level Chebyshev step and CG product (same hierarchy, inputs and launch shapes)
    def profiled(n_steps, **opts):
        h.profile(True)
        outs_p = [step(**opts)[1] for _ in range(n_steps)]
        n_cheb, ms_cheb = h.profile_query(regmg.TIMED_CHEB)
        n_cg, ms_cg = h.profile_query(regmg.TIMED_CG_MATVEC)
        h.profile(False)
        return n_cheb, ms_cheb / max(n_cheb, 1), n_cg, ms_cg / max(n_cg, 1), outs_p[-1]

    n_cheb, avg_cheb, n_cg, avg_cg, prof_out = profiled(args.profile_steps)
    print(f"[bench] profiled pass: Chebyshev step {avg_cheb * 1e3:.1f} us over {n_cheb} launches",
          file=sys.stderr, flush=True)
    info0 = h.level_info(0)
    rows = info0["n_regional"]
    lk = h.level_kernel(0)
    tiles = h.level_tiles(0)
    table_regions = h.level_table_regions(0)
    tiled = lk["kernel"] in (1, 2)  # the 2.5D kernel computes D^-1 of one-region rows

    def stored_bytes_per_row(table):
        bpr = float(cheb_bytes_per_row(lk["coefs"], not tiled))
        if table:
            # every region served: every coupling comes from the regions' class tables
            bpr -= 8 * lk["coefs"]
        return bpr

    stored_bpr = stored_bytes_per_row(table_regions == w.nreg)
    achieved = stored_bpr * rows / (avg_cheb * 1e-3) / 1e9
    method_bpr = METHOD_CHEB_BYTES_PER_ROW
    achieved_cg = cg_matvec_bytes_per_row(ALGO_COEFS) * rows / (avg_cg * 1e-3) / 1e9
    traffic, traffic_sha = counted_traffic()
    if args.workload != "c2" or traffic_sha != kernel_source_sha():
        traffic = None
    general = None
    if table_regions:
        # the general path: the same operator and tiles with every coupling streamed
        n0, avg0, _, _, out0 = profiled(1, region_table=0)
        bpr0 = stored_bytes_per_row(False)
        general = {
            "kernel": "k_stencil3d<Cheb, half stencil> (region_table = 0: all 14 upper couplings streamed)",
            "bytes_per_row": bpr0,
            "avg_launch_ms": avg0,
            "launches": n0,
            "achieved": bpr0 * rows / (avg0 * 1e-3) / 1e9,
            "frac": bpr0 * rows / (avg0 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "solve_ms": out0["solve_ms"],
            "iterations": out0["iterations"],
        }
    h.close()

    line = {
        "metric": METRIC,
        "value": float(np.median(solves)),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("3D Q1 Laplacian 27-point, 4x4x4 regions of 82^3 nodes (composite 325^3), FP64, "
                         "4-level regional V-cycle, Chebyshev degree 3, PCG to 1e-8, rhs U[-1,1] seed 0"
                         if args.workload == "c2" else args.workload),
            "regional_rows": rows,
            "table_regions": table_regions,
            "tiles": tiles,
            "iterations": last["iterations"],
            "true_relres": last["true_relres"],
            "setup_s_median": float(np.median(setups)),
            "solve_s_per_step": solves,
            "step": "device assembly + hierarchy setup + PCG solve",
            "kernel_launches_per_solve": launches,
            "cg_matvec_gbs_method_bytes": achieved_cg,
            # device ms of each region level's share of the preconditioner (profiled pass)
            "level_ms": prof_out["level_ms"][:w.nlevels],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_stencil_table<Cheb> (finest-level fused Chebyshev step, whole-row 2.5D tiles, every "
                       "coupling from the regions' class tables)"
                       if table_regions == w.nreg else
                       "k_stencil3d<Cheb, half stencil> (finest-level fused Chebyshev step, 2.5D tiles, upper "
                       "half of the symmetric stencil streamed)" if lk["coefs"] == 14 else
                       "k_stencil3d<Cheb> (finest-level fused Chebyshev step, 2.5D tiles)"),
            # the bytes this kernel must move per row: u, b, d read, d, u written, D^-1 of shared rows,
            # and the upper couplings of rows whose region the class tables do not serve
            "bytes_per_row": round(stored_bpr, 2),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "counted_hbm_gbs": traffic / (avg_cheb * 1e-3) / 1e9 if traffic else None,
            "bytes_per_launch": stored_bpr * rows,
            "avg_launch_ms": avg_cheb,
            "launches": n_cheb,
            "timing": "HIP events around each launch, in a profiled pass after the timed steps",
            # the method's own step streams the whole 27-point operator (264 B/row): the rate this
            # step runs at in those terms (above the HBM peak where the table spares the stream)
            "method_bytes_per_row": method_bpr,
            "method_equivalent_gbs": method_bpr * rows / (avg_cheb * 1e-3) / 1e9,
            "general_path": general,
            "copy_gbs": copy_rate_gbs(),
        },
    }
    if not args.no_variants and args.workload == "c2":
        line["variants"] = {
            "mixed_precision": variant_mixed(dev),
            "batched": variant_batched(dev),
            "learned_interpolation": variant_learned(dev),
            "graph_2d": variant_graph_2d(dev),
            "noninvasive_csr": variant_noninvasive(dev),
            "mg_as_solver": variant_mg_solver(dev),
            "hybrid_table5": variant_hybrid(dev),
            "coarse_amg": variant_coarse_amg(dev),
        }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(last["iterations"], rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
