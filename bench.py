#!/usr/bin/env python3
"""Benchmark of the flux-stencil hot path on one MI355X.

One step = the whole path over one batch of input already resident in HBM:
  build (face enumeration, path-radius neighbour rows, binning by row count, row
  assembly, weighted least-squares solve per face) followed by the operator apply
  L(Phi) (face-flux gather and divergence).
Workload: the 3D fourth-order case -- unit cube minus the sphere of radius 0.3 centred
at (0.5, 0.5, 0.5) on a 64^3 grid, 35 monomials, path radius 3, Dirichlet boundaries,
Phi ~ N(0, 1) (seed 2).  Inputs are synthetic: the moments come from host quadrature of
the level set (cutgeom), done before the timed region.

Prints one JSON line (stdout).  Progress goes to stderr.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cut-face stencils/s (3D, order 4, FP64) + L(phi) apply GB/s at 1e-11 rel err"
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector (= FP64 matrix) peak
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1411_4283_amd/csrc/stencil.hip", "paper_1411_4283_amd/csrc/stencil_impl.hpp",
                  "paper_1411_4283_amd/csrc/rows.hpp", "paper_1411_4283_amd/csrc/rows_dd.hpp",
                  "paper_1411_4283_amd/csrc/dd.hpp", "paper_1411_4283_amd/csrc/stencil_qr.hip",
                  "paper_1411_4283_amd/csrc/stencil_qr.hpp",
                  "paper_1411_4283_amd/csrc/common.hpp", "paper_1411_4283_amd/csrc/kernels.hpp",
                  "paper_1411_4283_amd/csrc/apply.hip", "paper_1411_4283_amd/csrc/gather.hpp")
TRAFFIC_FILE = "profiles/traffic_3d_order4_sphere64.md"


def sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per build of the stencil solves and per apply, from the rocprofv3 byte
    counters recorded in profiles/ -- only while the kernel sources are the ones measured
    (the summary records their SHA-256); otherwise None."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic:"):
                for kv in line[len("traffic:"):].split():
                    k, v = kv.split("=")
                    vals[k] = v
    if vals.get("sources_sha256") != sources_sha256():
        return None
    return {k: float(v) for k, v in vals.items() if k != "sources_sha256"}


def qr_flops(N, M):
    """Householder QR of an N x M matrix (LAPACK count)."""
    return 2 * N * M * M - 2.0 / 3.0 * M**3


def stream_copy_gbps(torch, dev, nbytes=1 << 30, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes / time), median of reps."""
    import numpy as np

    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del src, dst
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def householder_flops(N, M, T):
    """Per-face flop count of a backward-stable weighted least-squares stencil solve
    (LAPACK counts): Householder QR of the N x M weighted matrix, row assembly with T
    binomial terms per row, the minimum-norm solve and the weighting."""
    return (2 * N * M * M - 2.0 / 3.0 * M**3) + 2 * N * T + 2 * N * M + M * M + (4 * N * M - 2 * M * M) + N


def workload(name):
    import cutgeom as cg

    if name == "c3":
        return dict(shape=cg.ball_outside((0.5, 0.5, 0.5), 0.3), n=64, Q=4, R=3, seed=2,
                    desc="3D order 4: 64^3 unit cube minus sphere r=0.3 at (0.5,0.5,0.5), path radius 3, "
                         "35 monomials, Dirichlet, phi ~ N(0,1) seed 2")
    if name == "c4":
        return dict(n=48, Q=4, R=3, seed=3, n_geom=64,
                    desc="3D order 4, batched: 64 unit cubes minus spheres, centres 0.5 + U(-0.05,0.05)^3, "
                         "radii U(0.25,0.35) (default_rng(3): centres drawn first), 48^3 each, path radius 3, "
                         "35 monomials")
    if name == "c1":
        return dict(shape=cg.ball_outside((0.5, 0.5), 0.25), n=32, Q=2, R=2, seed=2,
                    desc="2D order 2: 32^2 unit square minus disk r=0.25, path radius 2, 6 monomials")
    raise SystemExit(f"unknown workload {name}")


def c4_shapes(w):
    import cutgeom as cg

    return cg.perturbed_spheres(w["n_geom"], w["seed"])


SCHEDULE_NOTE = ("per row-count bin (16 rows each): (XCD chunks, persistent workgroups per XCD or 0 for one per "
                 "face, split mode: 0 parts at their own narrower widths, 1 whole bin at its width, 2 part 0 "
                 "narrower, 3 parts 0-1 at width - 4), chosen by timing on the workload")


def batched_comparison(steps):
    """C4: all faces of 64 perturbed geometries in one build call (one launch per row-count
    bin across every geometry, autotuned schedule) versus one build call per geometry.
    Inputs are resident in HBM; each figure is the mean over `steps` builds."""
    import numpy as np
    import torch

    import cutgeom as cg
    import paper_1411_4283_amd as cc

    w = workload("c4")
    t0 = time.perf_counter()
    hosts = [cg.make_geometry(s, w["n"], w["Q"]) for s in c4_shapes(w)]
    log(f"c4: {len(hosts)} geometries in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    dgs = [cc.DeviceGeometry.from_host(h, dev) for h in hosts]
    del hosts

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n * 1e3

    # one build call per geometry (each with its own launches, default schedule)
    singles = [cc.Builder(dg, w["R"]) for dg in dgs]
    outs = [b.allocate() for b in singles]
    n_face = sum(b.sizes.n_face for b in singles)
    nnz = sum(b.sizes.nnz for b in singles)
    ms_single = timed(lambda: [b.build(out=o) for b, o in zip(singles, outs)], steps)
    ref = [o.val[: o.sizes.nnz].clone() for o in outs[:2]]
    del outs, singles
    torch.cuda.empty_cache()
    # the whole batch in one call: default schedule, then autotuned
    bb = cc.Builder(dgs, w["R"])
    st = bb.allocate()
    assert st.sizes.n_face == n_face and st.sizes.nnz == nnz
    ms_batch = timed(lambda: bb.build(out=st), steps)
    tuning, best = bb.autotune(out=st)
    ms_tuned = timed(lambda: bb.build(out=st), steps)
    # the batch holds the same stencils as the separate builds (first two geometries)
    off = 0
    for r in ref:
        assert torch.equal(st.val[off: off + r.numel()], r), "batched stencils differ from per-geometry ones"
        off += r.numel()
    sched = [(int(tuning.xcd_chunks[b]), int(tuning.blocks_per_xcd[b]), int(tuning.split[b])) for b in range(8)]
    flagged = int((st.status[: st.sizes.n_face] != 0).sum())
    out = {"workload": w["desc"], "n_geom": len(dgs), "n_face": int(n_face), "nnz": int(nnz),
           "per_geometry_ms": ms_single, "batched_ms": ms_batch, "batched_autotuned_ms": ms_tuned,
           "per_geometry_faces_per_s": n_face / (ms_single * 1e-3),
           "batched_autotuned_faces_per_s": n_face / (ms_tuned * 1e-3),
           "speedup_vs_per_geometry": ms_single / ms_tuned,
           "schedule_per_bin": sched, "schedule_note": SCHEDULE_NOTE, "bin_best_ms": best,
           "faces_flagged": flagged, "faces_by_qr": int(st.qr_faces),
           "parity_note": "stencils against the oracle on 8 seeded geometries of this batch (targeted faces): "
                          "tests/test_gpu_parity.py::test_batched_perturbed_spheres_against_oracle"}
    del st, bb, dgs
    torch.cuda.empty_cache()
    return out


def regular_face_count(g, R):
    """Faces between two cells whose whole L1 ball of radius R consists of full interior
    cells with all faces open (the neighbour search's fixed-row case); host numpy."""
    import numpy as np

    n = g.n[0]
    vol = (g.kappa > 0).reshape(n, n, n)
    eb = np.zeros(g.ncell, bool)
    eb[g.eb_cell] = True
    eb = eb.reshape(n, n, n)
    a0 = g.face_mom[0][:, 0].reshape(n, n, n + 1)
    a1 = g.face_mom[1][:, 0].reshape(n, n + 1, n)
    a2 = g.face_mom[2][:, 0].reshape(n + 1, n, n)
    opn = (a0[:, :, :-1] > 0) & (a0[:, :, 1:] > 0) & (a1[:, :-1] > 0) & (a1[:, 1:] > 0) & (a2[:-1] > 0) & (a2[1:] > 0)
    r = vol & ~eb & opn
    for ax in range(3):
        idx = [slice(None)] * 3
        for e in (0, -1):
            idx[ax] = e
            r[tuple(idx)] = False
    for _ in range(R):
        r2 = r.copy()
        r2[1:-1, 1:-1, 1:-1] &= (r[:-2, 1:-1, 1:-1] & r[2:, 1:-1, 1:-1] & r[1:-1, :-2, 1:-1] & r[1:-1, 2:, 1:-1]
                                 & r[1:-1, 1:-1, :-2] & r[1:-1, 1:-1, 2:])
        r = r2
    return int((r[:, :, :-1] & r[:, :, 1:]).sum() + (r[:, :-1] & r[:, 1:]).sum() + (r[:-1] & r[1:]).sum())


def adjoint_timings(torch, cc, b, st, phi, flux, reps=5):
    """The adjoints on the same stencils: the transpose, the apply adjoint (Phi-bar, val-bar,
    scale-bar) and the stencil backward with a cotangent on every face.  HIP events on the
    launch stream, median of `reps` after one warm-up."""
    import numpy as np

    s = st.sizes
    dev = phi.device

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def transpose():
        st.transpose = None
        cc.build_transpose(st)

    t_tr = timed(transpose)
    lbar = torch.from_numpy(np.random.default_rng(8).standard_normal(s.n_vol)).to(dev)
    t_adj = timed(lambda: cc.apply_adjoint(st, lbar, phi=phi, flux=flux))
    # algorithmic bytes of the apply adjoint: the CSC (nz, nz_face) and val through it, the
    # CSR (col, val-bar written) with Phi, face cotangents, Phi-bar, and per volume its face
    # table, scale, lbar, flux terms and scale-bar
    b_adj = (4 + 4 + 8) * s.nnz + (4 + 8) * s.nnz + 8 * (2 * s.n_phi + 2 * s.n_face) + (4 * 7 + 8 * 3) * s.n_vol
    vb = torch.from_numpy(np.random.default_rng(9).standard_normal(s.nnz)).to(dev)
    sb = torch.from_numpy(np.random.default_rng(10).standard_normal(s.n_vol)).to(dev)
    t_bw = timed(lambda: b.backward(st, vb, sb))
    return {"transpose_ms": t_tr, "apply_adjoint_ms": t_adj, "apply_adjoint_bytes": b_adj,
            "apply_adjoint_gbps": b_adj / (t_adj * 1e-3) / 1e9,
            "stencil_backward_ms": t_bw, "stencil_backward_faces_per_s": s.n_face / (t_bw * 1e-3),
            "note": "stencil backward with a cotangent on every face (rebuilds each face's system); "
                    "includes the per-Phi-entry moment reduction"}


_ORACLE_STATE = {}


def reuse_timings(torch, cc, dg, R, tuning, st_full, steps, n_face, full_ms):
    """The build with template reuse (faces whose systems are bitwise identical copy one
    solved face's stencil), same schedule, timed like the main step; its output is
    compared with the full build bit for bit.  Reported beside the headline, which solves
    every face as the paper does."""
    from paper_1411_4283_amd import _lib

    br = cc.Builder(dg, R, reuse_templates=True)
    br.set_tuning(tuning)
    br.query()
    sr = br.allocate()
    for _ in range(2):
        br.build(out=sr)
    torch.cuda.synchronize()
    _lib.set_profiling(True)
    solve = []
    t0 = time.perf_counter()
    for _ in range(steps):
        br.build(out=sr)
        solve.append(_lib.last_profile()["solve"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.set_profiling(False)
    ms = (t1 - t0) / steps * 1e3
    same = all(torch.equal(getattr(sr, k), getattr(st_full, k)) for k in ("row_ptr", "col", "val", "status"))
    return {"ms_per_step": ms, "faces_per_s": n_face / (ms * 1e-3), "speedup_vs_full_build": full_ms / ms,
            "solve_ms": sum(solve) / len(solve), "faces_copied": int(sr.reused), "faces_solved": int(n_face - sr.reused),
            "bitwise_equal_to_full_build": bool(same), "packed_apply": packed_apply_timings(torch, cc, sr)}


def packed_apply_timings(torch, cc, st, reps=20):
    """The compressed stencils (template copies as a slot plus run bases) against the plain
    CSR apply on the same stencils: HIP events on the launch stream, median of `reps`
    each, outputs compared bit for bit.  Algorithmic bytes as for the plain apply, with
    each packed face's entries replaced by its face, slot and run bases, plus the face
    phases, the list of CSR faces and the slot tables."""
    import numpy as np

    s = st.sizes
    dev = st.val.device
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    pk = cc.pack(st)
    torch.cuda.synchronize()
    pack_ms = (time.perf_counter() - t0) * 1e3
    phi = torch.from_numpy(np.random.default_rng(2).standard_normal(s.n_phi)).to(dev)
    lphi, flux = cc.apply(st, phi)
    lphi2, flux2 = cc.apply_packed(st, pk, phi)

    def med(fn):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, z in ev:
            a.record(stream)
            fn()
            z.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(z) for a, z in ev]))

    plain_ms = med(lambda: cc.apply(st, phi, lphi, flux))
    packed_ms = med(lambda: cc.apply_packed(st, pk, phi, lphi2, flux2))
    same = torch.equal(lphi, lphi2) and torch.equal(flux, flux2)
    rp = st.row_ptr.cpu().numpy()
    flag = pk.flag[: s.n_face].cpu().numpy().astype(bool)
    nnz_packed = int(np.sum(np.diff(rp)[flag]))
    common = 8 * (s.n_face + 1) + 8 * s.n_phi + 16 * s.n_vol
    plain_bytes = 12 * s.nnz + common
    packed_bytes = 12 * (s.nnz - nnz_packed) + pk.bytes_per_apply() + common
    return {"ms": packed_ms, "plain_apply_ms_same_stencils": plain_ms, "speedup_vs_plain_apply": plain_ms / packed_ms,
            "bytes_per_launch": int(packed_bytes), "plain_bytes_per_launch": int(plain_bytes),
            "gbps": packed_bytes / (packed_ms * 1e-3) / 1e9, "frac_of_hbm_peak": packed_bytes / (packed_ms * 1e-3)
            / 1e9 / PEAK_HBM_GBS, "faces_packed": int(pk.sizes.n_packed), "entries_packed": nnz_packed,
            "slots": int(pk.sizes.n_slot), "max_runs": int(pk.sizes.max_runs), "pack_ms": pack_ms,
            "bitwise_equal_to_plain_apply": bool(same),
            "note": "kernels k_apply_packed (CSR groups with packed faces skipped, then the packed faces) + "
                    "k_divergence"}


def laplacian_timings(torch, cc, st, phi, face_apply_ms, reps=20):
    """The operator as one matrix over volumes: its build (merge of each volume's face
    rows) and its apply (one gather per volume), HIP events on the launch stream, median
    of `reps`; algorithmic bytes as for the face apply (entries 12 B, row offsets, Phi and
    the output once)."""
    import numpy as np

    stream = torch.cuda.current_stream()

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    holder = {}
    build_ms = timed(lambda: holder.__setitem__("lap", cc.build_laplacian(st)), 5)
    lap = holder["lap"]
    lphi = torch.empty(max(st.sizes.n_vol, 1), dtype=torch.float64, device=phi.device)
    ms = timed(lambda: cc.apply_laplacian(lap, phi, lphi), reps)
    s = st.sizes
    nbytes = 12 * lap.nnz + 8 * (s.n_vol + 1) + 8 * s.n_phi + 8 * s.n_vol
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"nnz": int(lap.nnz), "face_nnz": int(s.nnz), "build_ms": build_ms, "apply_ms": ms,
           "bytes_per_launch": nbytes, "apply_gbps": gbs,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": gbs / PEAK_HBM_GBS, "kernel": "k_flux over volume rows"},
           "speedup_vs_face_apply": face_apply_ms / ms}
    return out, lap


def weight_study(torch, cc, powers=(0.0, 2.0, 3.0, 4.0, 5.0, 6.0, 8.0)):
    """Sec. 2.4's weights W = (2d)^-p beyond half a cell, p swept on the paper's spectrum
    case (64 x 64 grid outside the circle r = 0.25, fourth order, path radius 3, Dirichlet):
    per p, the rightmost and leftmost eigenvalues from GPU Arnoldi (cutcell_ritz: 60 steps
    on A, 20 shift-invert steps) and the L1 solution error of the GPU solve for the paper's
    2D exact solution.  The paper uses p = 5."""
    import numpy as np

    import cutgeom as cg

    g = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.25), 64, 4)
    tp = 2 * math.pi
    I = g.integrate(cg.trig_product((tp, tp), (-tp * math.sqrt(2) / 2, -tp * math.sqrt(3) / 2)))
    hD, hD1 = g.h**2, g.h
    kap = g.kappa
    vol_avg = np.divide(I["vol_int"], kap * hD, out=np.zeros_like(kap), where=kap > 0)
    face_avg = [np.divide(I["face_int"][d], g.alpha(d) * hD1, out=np.zeros(len(g.alpha(d))), where=g.alpha(d) > 0)
                for d in range(2)]
    phi = g.layout_phi(vol_avg, I["eb_int"] / (g.eb_mom[:, 0] * hD1), face_avg)
    vols = np.nonzero(kap > 0)[0]
    rhs = I["vol_lap"][vols] / (kap[vols] * hD)
    V = kap[vols] * hD
    dev = torch.device("cuda:0")
    dg = cc.DeviceGeometry.from_host(g, dev)
    phi_t = torch.from_numpy(phi).to(dev)
    rhs_t = torch.from_numpy(rhs).to(dev)
    rows = []
    t0 = time.perf_counter()
    for p in powers:
        st = cc.Builder(dg, 3, weight_power=p).build()
        r0, e0, ok0 = cc.ritz(st, mode=0, steps=60)
        r1, e1, ok1 = cc.ritz(st, mode=1, steps=20, inner_rtol=1e-10)
        conv0 = r0[e0 <= 1e-6]
        res = cc.solve(st, phi_t, rhs_t, rtol=1e-13, restart=200, max_iters=4000)
        e = res.x.cpu().numpy() - phi[: len(vols)]
        # shift-invert converges to the eigenvalue nearest 0 (largest |theta| of A^-1); Arnoldi
        # on A to the largest in magnitude
        near0 = r1[np.argmin(np.abs(r1))] if ok1 and len(r1) else None
        rows.append({"p": p, "lambda_nearest_zero": None if near0 is None else float(near0.real),
                     "lambda_min": float(r0.real.min()),
                     "max_re_converged_ritz_of_A": float(conv0.real.max()) if len(conv0) else None,
                     "ritz_converged": bool(ok0 and ok1),
                     "solve_converged": bool(res.converged), "solve_iterations": res.iters,
                     "error_L1": float(np.sum(np.abs(e) * V) / V.sum()), "error_Linf": float(np.abs(e).max()),
                     "flagged_faces": int(st.status.ne(0).sum())})
        log(f"weight p={p}: {rows[-1]}")
    return {"case": "64x64 outside circle r=0.25, order 4, path radius 3, Dirichlet", "rows": rows,
            "seconds": time.perf_counter() - t0}


def spectrum_at_scale(cc, st, lap):
    """Rightmost and leftmost eigenvalues of the workload's operator (GPU Arnoldi through
    the volume matrix)."""
    t0 = time.perf_counter()
    import numpy as np

    r1, e1, ok1 = cc.ritz(st, mode=1, steps=20, lap=lap, inner_rtol=1e-10)
    r0, e0, ok0 = cc.ritz(st, mode=0, steps=60, lap=lap)
    near0 = r1[np.argmin(np.abs(r1))]
    conv0 = r0[e0 <= 1e-6]
    return {"lambda_nearest_zero": float(near0.real), "lambda_nearest_zero_residual": float(e1[np.argmin(np.abs(r1))]),
            "lambda_min": float(r0.real.min()), "lambda_min_residual": float(e0[np.argmin(r0.real)]),
            "max_re_converged_ritz_of_A": float(conv0.real.max()) if len(conv0) else None,
            "max_re_any_ritz_of_A": float(r0.real.max()), "converged": bool(ok0 and ok1),
            "seconds": time.perf_counter() - t0,
            "method": "Arnoldi: 20 shift-invert steps (GMRES inner solves, rtol 1e-10) for the eigenvalue nearest 0, "
                      "60 steps on A for the most negative"}


def solve_timings(torch, cc, g, st, apply_ms, rtol=1e-12, restart=50, lap=None):
    """The discrete Poisson problem on the workload's geometry (Dirichlet data and source
    from the paper's 3D exact solution, Sec. 3.6) solved by the GPU GMRES (cutcell_solve);
    wall-clock time of the call, iterations, and the solution error against the exact
    volume averages."""
    import numpy as np

    import cutgeom as cg

    tp = 2 * math.pi
    I = g.integrate(cg.trig_product((tp,) * g.D, (-tp * math.sqrt(2) / 2, -tp * math.sqrt(3) / 2, -tp * 0.54321)[: g.D]))
    hD, hD1 = g.h**g.D, g.h ** (g.D - 1)
    kap = g.kappa
    vol_avg = np.divide(I["vol_int"], kap * hD, out=np.zeros_like(kap), where=kap > 0)
    eb_avg = I["eb_int"] / (g.eb_mom[:, 0] * hD1)
    face_avg = [np.divide(I["face_int"][d], g.alpha(d) * hD1, out=np.zeros(len(g.alpha(d))), where=g.alpha(d) > 0)
                for d in range(g.D)]
    phi = g.layout_phi(vol_avg, eb_avg, face_avg)
    vols = np.nonzero(kap > 0)[0]
    rhs = I["vol_lap"][vols] / (kap[vols] * hD)
    dev = st.val.device
    phi_t = torch.from_numpy(phi).to(dev)
    rhs_t = torch.from_numpy(rhs).to(dev)
    cc.solve(st, phi_t, rhs_t, rtol=rtol, restart=restart, max_iters=5, lap=lap)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = cc.solve(st, phi_t, rhs_t, rtol=rtol, restart=restart, max_iters=20000, lap=lap)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    e = res.x.cpu().numpy() - phi[: len(vols)]
    V = kap[vols] * hD
    # algorithmic bytes of the Arnoldi steps: the matvec (the volume matrix's or the face
    # path's bytes) and, at Krylov index j, two Gram-Schmidt passes each reading j+1 basis
    # vectors twice (inner products, update) and w three times, plus the scaling of D^-1 v
    n = len(vols)
    s = st.sizes
    mv = (12 * lap.nnz + 8 * (n + 1) + 8 * s.n_phi + 8 * n) if lap is not None else \
        (12 * s.nnz + 8 * (s.n_face + 1) + 8 * s.n_phi + 16 * n)
    steps_bytes = 0
    for it in range(res.iters):
        j = it % restart
        steps_bytes += mv + 2 * (8 * n * 2 * (j + 1) + 8 * n * 3) + 8 * n * 5
    gbs = steps_bytes / (ms * 1e-3) / 1e9
    return {"ms": ms, "iterations": res.iters, "ms_per_iteration": ms / max(res.iters, 1), "relres": res.relres,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "bytes": steps_bytes,
                         "note": "algorithmic bytes of all Arnoldi steps over the whole solve time"},
            "converged": res.converged, "rtol": rtol, "restart": restart,
            "apply_share": res.iters * apply_ms / ms, "n_vol": int(len(vols)),
            "error_Linf": float(np.abs(e).max()), "error_L1": float(np.sum(np.abs(e) * V) / V.sum()),
            "preconditioner": "Jacobi (right)", "matvec": "volume matrix" if lap is not None else "face fluxes"}


def _oracle_chunk(faces, keep=None):
    """Worker: the oracle's stencil + face flux for a list of faces (one thread).  With a
    dict `keep`, the stencils are stored in it by face."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    g, en, R, phi = (_ORACLE_STATE[k] for k in ("g", "en", "R", "phi"))
    with threadpool_limits(limits=1):
        for f in faces:
            idx, sv, st = oracle.face_stencil(g, en, int(f), R)
            _ = float(np.dot(sv, phi[idx]))
            if keep is not None:
                keep[int(f)] = (sv, int(st))
    return len(faces)


def _cond_chunk(faces):
    """Worker: condition numbers of the column-equilibrated W A of a list of faces."""
    from threadpoolctl import threadpool_limits

    import oracle

    g, en, R = (_ORACLE_STATE[k] for k in ("g", "en", "R"))
    with threadpool_limits(limits=1):
        return [oracle.face_condition(g, en, int(f), R) for f in faces]


def cpu_baseline(g, R, sample, seed=7, workers=None):
    """The oracle (numpy, extended-precision Householder QR per face) on a random sample of
    faces: build (neighbours, rows, weights, stencil) plus each face's flux in the apply, and
    the enumeration pro rata.  One thread, and (if `workers` > 1) the same per-face work
    spread over that many forked worker processes, which also compute the sample's
    condition numbers.  Runs before the GPU is touched.  Returns the result dict and
    (faces, their oracle stencils, their condition numbers or None)."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        en = oracle.enumerate_geometry(g)
        t_enum = time.perf_counter() - t0
    faces = np.random.default_rng(seed).choice(en.n_face, min(sample, en.n_face), replace=False)
    phi = np.random.default_rng(2).standard_normal(en.n_phi)
    _ORACLE_STATE.update(g=g, en=en, R=R, phi=phi)
    kept = {}
    t0 = time.perf_counter()
    _oracle_chunk(faces, kept)
    t_faces = time.perf_counter() - t0
    t = t_faces + t_enum * len(faces) / en.n_face
    out = dict(value=len(faces) / t, unit="faces/s", cores=1, kind="oracle",
               sample=f"{len(faces)} faces drawn uniformly (seed {seed}) of {en.n_face}; stencil build + "
                      f"face flux per face, enumeration pro rata; {t:.1f} s on one thread")
    conds = None
    if workers and workers > 1:
        many = np.random.default_rng(seed + 1).choice(en.n_face, min(4 * sample, en.n_face), replace=False)
        chunks = np.array_split(many, 8 * workers)
        pool = mp.get_context("fork").Pool(workers)
        try:
            t0 = time.perf_counter()
            done = sum(pool.map(_oracle_chunk, chunks))
            tw = time.perf_counter() - t0
            # condition numbers of the timed sample's systems (not timed), for the parity report
            conds = np.concatenate([np.asarray(c) for c in pool.map(_cond_chunk, np.array_split(faces, 4 * workers))])
        finally:
            # every worker exits and is reaped before the GPU is touched
            pool.close()
            pool.join()
        out["all_cores"] = dict(value=done / tw, unit="faces/s", cores=workers,
                                sample=f"{done} faces (seed {seed + 1}) over {workers} processes, {tw:.1f} s; "
                                       "enumeration not included")
    out["host"] = host_info()
    return out, (faces, kept, conds)


def parity_report(st, ref):
    """The timed build's stencils on the oracle's timed sample of faces: worst relative error
    per face (max over the row against the row's largest oracle value), status agreement,
    and the condition numbers of those faces' equilibrated W A."""
    import numpy as np

    faces, kept, conds = ref
    rp = st.row_ptr.cpu().numpy()
    val = st.val.cpu().numpy()
    status = st.status.cpu().numpy()
    worst, wf, mism = 0.0, -1, 0
    for f in faces:
        f = int(f)
        sv, so = kept[f]
        if status[f] != so:
            mism += 1
            continue
        if so != 0:
            continue
        err = float(np.abs(val[rp[f]:rp[f + 1]] - sv).max() / np.abs(sv).max())
        if err > worst:
            worst, wf = err, f
    out = {"faces": int(len(faces)), "worst_rel_err": worst, "worst_face": wf, "status_mismatches": mism,
           "bar": 1e-11}
    if conds is not None:
        out["cond"] = {f"p{q}": float(np.percentile(conds, q)) for q in (50, 90, 99)}
        out["cond"]["max"] = float(np.max(conds))
        if wf >= 0:
            out["cond_of_worst_face"] = float(conds[list(map(int, faces)).index(wf)])
    return out


def qr_all_timings(torch, cc, dg, R, st_ref, n_face, flops, reps=2):
    """The same build with every face solved by Householder QR (double-double rows and
    refinement residuals): time per build and its stencils against the default build's."""
    b = cc.Builder(dg, R, factorization="qr")
    st = b.allocate()
    b.build(out=st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.build(out=st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    nnz = int(st.sizes.nnz)
    rp = st_ref.row_ptr
    face = torch.repeat_interleave(torch.arange(n_face, device=rp.device), rp[1:] - rp[:-1])
    diff = (st.val[:nnz] - st_ref.val[:nnz]).abs()
    dmax = torch.zeros(n_face, dtype=torch.float64, device=rp.device).scatter_reduce_(0, face, diff, "amax")
    smax = torch.zeros(n_face, dtype=torch.float64, device=rp.device).scatter_reduce_(0, face,
                                                                                       st_ref.val[:nnz].abs(), "amax")
    ok = smax > 0
    rel = float((dmax[ok] / smax[ok]).max())
    same_status = bool(torch.equal(st.status[:n_face], st_ref.status[:n_face]))
    del b, st, face, diff, dmax, smax
    torch.cuda.empty_cache()
    return {"ms_per_build": ms, "faces_per_s": n_face / (ms * 1e-3), "tflops_lapack_count": flops / (ms * 1e-3) / 1e12,
            "max_rel_diff_vs_default_build": rel, "same_status": same_status,
            "note": "every face by the QR path (one wave per face, factors in shared memory, the exact B in a "
                    "workspace slot, double-double rows and "
                    "residuals); the default build routes only ill-conditioned faces there"}


def host_info():
    """The host the oracle ran on: logical CPUs and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"logical_cpus": os.cpu_count(), "cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-sample", type=int, default=4000, help="faces of the oracle's timed sample (~12 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-geometry comparison")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip timing the adjoints")
    ap.add_argument("--no-reuse", action="store_true", help="skip timing the template-reuse build")
    ap.add_argument("--no-solve", action="store_true", help="skip timing the GPU Poisson solve")
    ap.add_argument("--no-laplacian", action="store_true", help="skip the volume-matrix build and apply")
    ap.add_argument("--no-weight-study", action="store_true", help="skip the weight-exponent study and spectra")
    ap.add_argument("--no-qr-all", action="store_true", help="skip timing the build with every face by QR")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one 256 MiB device copy (reference kernel for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import cutgeom as cg

    w = workload(args.workload)
    t0 = time.perf_counter()
    g = cg.make_geometry(w["shape"], w["n"], w["Q"])
    log(f"geometry {time.perf_counter() - t0:.2f} s")
    base = None
    if not args.no_cpu_baseline:
        # before anything initialises the GPU: the worker processes are forks of this one
        log("cpu baseline (oracle)")
        base, parity_ref = cpu_baseline(g, w["R"], args.cpu_sample, workers=min(16, os.cpu_count() or 1))
    regular = regular_face_count(g, w["R"]) if g.D == 3 else None

    import torch

    import paper_1411_4283_amd as cc
    from paper_1411_4283_amd import _lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    dg = cc.DeviceGeometry.from_host(g, dev)
    b = cc.Builder(dg, w["R"])
    s = b.query()
    st = b.allocate()
    phi = torch.from_numpy(np.random.default_rng(w["seed"]).standard_normal(s.n_phi)).to(dev)
    lphi = torch.empty(max(s.n_vol, 1), dtype=torch.float64, device=dev)
    flux = torch.empty(max(s.n_face, 1), dtype=torch.float64, device=dev)
    log(f"faces {s.n_face} nnz {s.nnz} phi {s.n_phi} max rows {s.max_rows}")
    schedule = None
    if not args.no_autotune:
        tuning, best = b.autotune(out=st)
        schedule = [(int(tuning.xcd_chunks[i]), int(tuning.blocks_per_xcd[i]), int(tuning.split[i]))
                    for i in range(8)]
        log(f"autotuned per bin (xcd chunks, blocks per xcd, split mode): {schedule}")

    for _ in range(args.warmup):
        b.build(out=st)
        cc.apply(st, phi, lphi, flux)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    _lib.set_profiling(True)
    solve_ms, apply_ms, phases = [], [], []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.build(out=st)
        prof = _lib.last_profile()
        solve_ms.append(prof["solve"])
        phases.append(prof)
        ev[k][0].record(stream)
        cc.apply(st, phi, lphi, flux)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.set_profiling(False)
    apply_ms = [a.elapsed_time(z) for a, z in ev]
    # the apply on its own: 3 warm-ups, median of 20 (HIP events on the launch stream)
    for _ in range(3):
        cc.apply(st, phi, lphi, flux)
    ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for a, z in ev2:
        a.record(stream)
        cc.apply(st, phi, lphi, flux)
        z.record(stream)
    torch.cuda.synchronize()
    apply_ms = [a.elapsed_time(z) for a, z in ev2]
    ms_per_step = (t1 - t0) / args.steps * 1e3
    log(f"ms/step {ms_per_step:.3f}  solve {np.mean(solve_ms):.3f} ms  apply {np.mean(apply_ms) * 1e3:.1f} us "
        f"({st.qr_faces} faces by QR)")

    rp = st.row_ptr.cpu().numpy()
    N = np.diff(rp)
    M = math.comb(w["Q"] + g.D, g.D)
    T = math.comb(w["Q"] + 2 * g.D, 2 * g.D)
    status = st.status.cpu().numpy()[: s.n_face]
    ok = status == 0
    flops = float(np.sum(householder_flops(N[ok].astype(np.float64), M, T)))
    flops_qr = float(np.sum(qr_flops(N[ok].astype(np.float64), M)))
    solve = float(np.mean(solve_ms))
    achieved_tf = flops / (solve * 1e-3) / 1e12
    apply_mean = float(np.median(apply_ms))
    copy_gbs = stream_copy_gbps(torch, dev)
    traffic = measured_traffic() if args.workload == "c3" else None
    if args.calibrate_copy:
        # an elementwise pass reading 256 MiB and writing 256 MiB, under a kernel name of
        # its own (torch's negation kernel)
        src = torch.empty(1 << 25, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    bytes_alg = 12 * s.nnz + 8 * (s.n_face + 1) + 8 * s.n_phi + 16 * s.n_vol
    apply_gbs = bytes_alg / (apply_mean * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": s.n_face / (ms_per_step * 1e-3),
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "grid": w["n"], "order": w["Q"], "path_radius": w["R"],
                   "n_face": int(s.n_face), "nnz": int(s.nnz), "n_phi": int(s.n_phi), "n_vol": int(s.n_vol)},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP64_TFLOPS,
                     "traffic": None if traffic is None else traffic["solve_bytes_per_build"],
                     "kernel": "k_stencil (all row-count bins)", "kernel_ms": solve,
                     "flops_per_launch": flops},
        "roofline_apply": {"bound": "hbm", "achieved": apply_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": apply_gbs / PEAK_HBM_GBS,
                           "traffic": None if traffic is None else traffic["apply_bytes"], "kernel": "k_flux + k_divergence",
                           "kernel_ms": apply_mean, "bytes_per_launch": bytes_alg},
        "apply_gbps": apply_gbs,
        "qr_only_tflops": flops_qr / (solve * 1e-3) / 1e12,
        "stream_copy_gbps": copy_gbs,
        "apply_frac_of_stream_copy": apply_gbs / copy_gbs,
        "build_faces_per_s": s.n_face / (float(np.mean([sum(v for v in p.values() if v > 0) for p in phases])) * 1e-3),
        "phases_ms": {k: float(np.mean([p[k] for p in phases])) for k in phases[0]},
        "schedule_per_bin": schedule,
        "schedule_note": SCHEDULE_NOTE,
        "faces_regular": regular,
        "faces_regular_note": "faces between two cells whose whole path-radius ball is plain interior volume "
                              "(fixed rows); every face, regular or not, is solved",
    }
    out["qr_faces"] = int(st.qr_faces)
    out["qr_faces_note"] = ("faces whose system the Gram path leaves to Householder QR (estimated cond of the "
                            "equilibrated W A above 3e4, a pivot ratio below 1e-4, or a refinement step above 1e-6 of the "
                            "stencil)")
    if base is not None:
        out["parity_sample"] = parity_report(st, parity_ref)
        log(f"parity sample: {out['parity_sample']}")
    if not args.no_qr_all:
        log("every face by Householder QR")
        out["qr_all"] = qr_all_timings(torch, cc, dg, w["R"], st, s.n_face, flops)
    if not args.no_adjoint:
        log("adjoint timings")
        out["adjoint"] = adjoint_timings(torch, cc, b, st, phi, flux)
    if not args.no_reuse:
        log("template reuse")
        out["template_reuse"] = reuse_timings(torch, cc, dg, w["R"], b.tuning, st, args.steps, s.n_face, ms_per_step)
    lap = None
    if not args.no_laplacian:
        log("volume matrix")
        out["laplacian"], lap = laplacian_timings(torch, cc, st, phi, apply_mean)
    if not args.no_weight_study:
        log("weight study and spectra")
        out["weight_study"] = weight_study(torch, cc)
        if lap is not None:
            out["spectrum_at_scale"] = spectrum_at_scale(cc, st, lap)
    if not args.no_solve:
        log("Poisson solve")
        out["poisson_solve"] = solve_timings(torch, cc, g, st, apply_mean)
        if lap is not None:
            out["poisson_solve_laplacian"] = solve_timings(torch, cc, g, st, out["laplacian"]["apply_ms"], lap=lap)
    del lap
    del st, b, dg
    torch.cuda.empty_cache()
    if not args.no_batched and args.workload == "c3":
        log("batched comparison (64 geometries)")
        out["batched"] = batched_comparison(max(1, min(args.steps, 3)))
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
