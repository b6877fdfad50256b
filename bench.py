"""Benchmark: Krylov block steps/s of the s-PKSM hot path at n = 1e6 on one MI355X.

One benchmark step = a forward solve of A X + X B = C1 C2^T and the adjoint solve
A^T L + L B^T = P1 P2^T with the same method, then the gradients of tr(P1^T X P2), on the
1000 x 1000 upwind convection-diffusion pair (n = 1e6, r = 4, k = 3, s = 8000,
nu = 1e-2, w_A = (1, 0.5), w_B = (-0.3, 1)).  Each solve runs a fixed window of d block
steps (tandem SpMM, truncated block Gram-Schmidt, sketch, sketched QR update), one
projected FP64 Sylvester solve with the residual estimate, the low-rank factorisation and
the stored-basis recovery.  `value` = tandem block steps (forward + adjoint) per second
of wall time over the whole step, inputs resident in HBM.

Also reported: the same step in plain FP64, the per-kernel roofline of the dominant
kernel family (HIP events inside the timed region), and the FP64 CPU oracle timed on a
bounded sample of the same workload.
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
WORKLOAD = "convdiff2d_1000"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--window", type=int, default=200, help="block steps per solve")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-tpksm", action="store_true", help="skip the t-PKSM comparison solve")
    ap.add_argument("--no-lyapunov", action="store_true", help="skip the Lyapunov comparison solve")
    ap.add_argument("--no-sorth", action="store_true",
                    help="skip the solve with the sketched-inner-product orthogonalisation")
    ap.add_argument("--no-srht", action="store_true", help="skip the solve with the subsampled randomized DCT")
    ap.add_argument("--concurrent", action="store_true",
                    help="run the forward and the adjoint solve of a step concurrently (two host threads, "
                         "one stream each)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="GiB: run only a plain device-to-device copy of this size (HBM counter calibration)")
    return ap.parse_args()


# Kernel sources whose change invalidates a stored counter measurement of the SpMM kernel.
SPMM_SOURCES = ["block_cgs.hip", "blockstep.hpp", "small_la.hpp"]
TRAFFIC_RECORD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                              "traffic_spmm_convdiff1000_r4_mixed.md")


def spmm_sources_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2311_16019_amd", "csrc")
    for name in SPMM_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, precision):
    """HBM bytes per launch from the committed counter record, or None when the record is
    missing, is for another kernel or precision, or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_RECORD) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if (rec.get("kernel") == kernel and rec.get("precision") == precision
                            and rec.get("sources_sha256") == spmm_sources_digest()):
                        return rec
    except OSError:
        pass
    return None


def copy_probe(gib):
    import torch
    nbytes = int(gib * (1 << 30)) // 8 * 8
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_probe_bytes=nbytes, copies=3)))


SELL_C = 64  # rows per slice of the sliced-ELL operator storage


def sell_bytes(M, w):
    """Bytes of one sweep over M in sliced-ELL form: padded entries (values + int32 columns)
    and the int32 slice offsets."""
    nnz_row = np.diff(M.indptr)
    ns = (M.shape[0] + SELL_C - 1) // SELL_C
    padded = np.zeros(ns * SELL_C, dtype=np.int64)
    padded[:M.shape[0]] = nnz_row
    entries = int(padded.reshape(ns, SELL_C).max(axis=1).sum()) * SELL_C
    return entries * (w + 4) + 4 * (ns + 1)


def algorithmic_bytes(family, cfg, w, d_avg):
    """Bytes one launch of a kernel family must move (both Krylov spaces), by its definition.

    w = bulk element size, blocks are n x r; k window blocks.  spmm: the operator in its
    sliced-ELL form streamed once (padded entries (w + 4) + 4 (slices + 1), the mean of the
    forward orientations A, B^T and the adjoint ones A^T, B), U_d read once, U~ written,
    the diagonal shift of A read.  dots: U~ and the k window blocks
    read.  update: U~ and the window read, U_{d+1} written.  sketch: U_{d+1} and the
    2-byte embedding table (zeta entries per row) read, s x r FP64 written.  whiten: the
    FP64 sketched basis Q (s x d r) read once.
    """
    n, r, s, k = cfg["n"], cfg["r"], cfg["s"], cfg["k"]
    blk = n * r * w
    if family == "spmm":
        a, b = cfg["A"].to_scipy(), cfg["B"].to_scipy()
        ops = [sell_bytes(M, w) for M in (a, b.T.tocsr(), a.T.tocsr(), b)]
        diag = 8 * n if cfg["sigma"] is not None else 0
        return (ops[0] + ops[1] + ops[2] + ops[3]) / 2 + 2 * (2 * blk) + diag
    per_space = {"dots": (1 + k) * blk, "update": (k + 2) * blk, "sketch": blk + 2 * 8 * n + 8 * s * r,
                 "whiten": 8 * s * r * d_avg}
    return 2 * per_space.get(family, 0)


def cpu_baseline(cfg, steps):
    """The FP64 oracle's tandem block steps/s on the same matrices (bounded sample)."""
    from oracle import sketch as osk
    from oracle.spksm import Space, as_operator
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    A = as_operator(cfg["A"])
    BT = as_operator(cfg["B"]).T.tocsr()
    sig = cfg["sigma"]
    su, sv = osk.space_seeds(cfg["sketch_seed"])
    SU = osk.sparse_sign(cfg["n"], cfg["s"], 8, su)
    SV = osk.sparse_sign(cfg["n"], cfg["s"], 8, sv)
    opu = (lambda X: A @ X) if sig is None else (lambda X: A @ X + sig[:, None] * X)
    U = Space(opu, SU, cfg["k"], cfg["r"], steps + 1, False)
    V = Space(lambda X: BT @ X, SV, cfg["k"], cfg["r"], steps + 1, False)
    U.init(cfg["C1"])
    V.init(cfg["C2"])
    t0 = time.perf_counter()
    for d in range(1, steps + 1):
        U.step(d)
        V.step(d)
    el = time.perf_counter() - t0
    return dict(value=steps / el, unit="tandem block steps/s", cores=int(threads), kind="oracle",
                sample=f"{steps} tandem block steps (d = 1..{steps}) of the FP64 oracle on the n = 1e6 "
                       f"convection-diffusion pair (SpMM, truncated MGS, QR, sketch, sketched QR update); "
                       f"{el:.1f} s; SciPy sparse products single-threaded, BLAS threads = {threads}")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    import torch

    import paper_2311_16019_amd as skr
    from workloads import make_config

    cfg = make_config(WORKLOAD)  # s = 8000 (4 * 500 * r), k = 3, r = 4, tol 1e-6
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    A = skr.Operator.from_csr(cfg["A"].indptr, cfg["A"].indices, cfg["A"].data, diag=cfg["sigma"])
    B = skr.Operator.from_csr(cfg["B"].indptr, cfg["B"].indices, cfg["B"].data)
    C1, C2, P1, P2 = dev(cfg["C1"]), dev(cfg["C2"]), dev(cfg["P1"]), dev(cfg["P2"])
    win = args.window

    def params(precision, profile=False):
        return dict(k=cfg["k"], maxit=win, p=win, s=cfg["s"], tol=cfg["tol"], seed=cfg["sketch_seed"],
                    precision=precision, recover="stored", profile=profile)

    wall = dict(forward=0.0, adjoint=0.0, grads=0.0, solves=0.0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]  # default priority
    pool = None
    if args.concurrent:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=2)

    def on_stream(st, fn, *a, **kw):
        with torch.cuda.stream(st):
            return fn(*a, stream=st, **kw)

    def one_step(precision, profile=False):
        prm = params(precision, profile)
        if pool is not None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ff = pool.submit(on_stream, streams[0], skr.solve, A, B, C1, C2, **prm)
            fa = pool.submit(on_stream, streams[1], skr.adjoint_solve, A, B, P1, P2, **prm)
            f, a = ff.result(), fa.result()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            g = skr.pairing_grads(f.X1, f.X2, C1, C2, P1, P2, L1=a.X1, L2=a.X2)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            wall["solves"] += 1e3 * (t2 - t0)
            wall["grads"] += 1e3 * (t3 - t2)
            return f, a, g
        t0 = time.perf_counter()
        f = skr.solve(A, B, C1, C2, **prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        a = skr.adjoint_solve(A, B, P1, P2, **prm)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g = skr.pairing_grads(f.X1, f.X2, C1, C2, P1, P2, L1=a.X1, L2=a.X2)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        wall["forward"] += 1e3 * (t1 - t0)
        wall["adjoint"] += 1e3 * (t2 - t1)
        wall["solves"] += 1e3 * (t2 - t0)
        wall["grads"] += 1e3 * (t3 - t2)
        return f, a, g

    # warm-up with every kernel family timed: the per-family table and the roofline kernel,
    # the single-kernel streaming family (spmm, dots, update) with the most time.  The timed
    # steps record events around that family's launches only (events around every launch of
    # every family lengthen the block steps by about a fifth).
    fam_warm = {}
    for _ in range(max(1, args.warmup)):
        f, a, _ = one_step(args.precision, profile=True)
        f_warm = f  # the comparison legs below time every family too, so they compare with this
        for res in (f, a):
            for k, (nl, ms) in res.kernels.items():
                L, M = fam_warm.get(k, (0, 0.0))
                fam_warm[k] = (L + nl, M + ms)
    single = [k for k in ("spmm", "dots", "update") if k in fam_warm]
    dominant = max(single, key=lambda k: fam_warm[k][1])

    torch.cuda.synchronize()
    for key in wall:
        wall[key] = 0.0
    t0 = time.perf_counter()
    fam = {}
    steps_done = 0
    split = dict(steps=0.0, proj=0.0, recover=0.0)
    last = None
    for _ in range(args.steps):
        f, a, g = one_step(args.precision, profile=dominant)
        for res in (f, a):
            steps_done += res.iters
            split["steps"] += res.ms_steps
            split["proj"] += res.ms_proj
            split["recover"] += res.ms_recover
            for k, (nl, ms) in res.kernels.items():
                L, M = fam.get(k, (0, 0.0))
                fam[k] = (L + nl, M + ms)
        last = (f, a, g)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1000.0 * el / args.steps
    value = steps_done / el

    f, a, g = last
    true_res = skr.true_residual(A, B, f.X1, f.X2, C1, C2)
    w = 4 if args.precision == "mixed" else 8
    nl, ms = fam[dominant]
    d_avg = (win + 1) / 2.0
    per_launch = algorithmic_bytes(dominant, cfg, w, d_avg)
    achieved = per_launch / (ms / nl * 1e-3) / 1e9
    rec = measured_traffic(dominant, args.precision)
    roofline = dict(kernel=dominant, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=int(rec["bytes_per_launch"]) if rec else None,
                    bytes_per_launch=int(per_launch), avg_launch_us=round(1000.0 * ms / nl, 2), launches=nl)
    families = {}  # from the warm-up step(s), every family timed
    for k, v in fam_warm.items():
        b = algorithmic_bytes(k, cfg, w, d_avg)
        families[k] = dict(launches=v[0], avg_us=round(1000.0 * v[1] / v[0], 2))
        if b:
            families[k]["gbs"] = round(b / (v[1] / v[0] * 1e-3) / 1e9, 1)

    out = dict(metric="Krylov tandem block steps/s at n=1M (forward + adjoint s-PKSM)", value=round(value, 2),
               unit="block steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 2),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64" if args.precision == "mixed"
               else "f64", data="synthetic",
               config=dict(workload="upwind convection-diffusion 1000x1000 pair (n=1e6), r=4, k=3, s=8000, "
                                    f"{win} block steps per solve, forward + adjoint, stored-basis recovery",
                           n=cfg["n"], r=cfg["r"], k=cfg["k"], s=cfg["s"], window=win, precision=args.precision),
               roofline=roofline, kernel_families=families,
               kernel_families_from="warm-up step, every kernel family timed (the timed steps time the roofline "
                                    "kernel's family only)",
               block_steps_per_s=round(steps_done / (split["steps"] * 1e-3), 1),
               time_split_ms=dict(block_steps=round(split["steps"] / args.steps, 2),
                                  projected_solves=round(split["proj"] / args.steps, 2),
                                  recovery=round(split["recover"] / args.steps, 2),
                                  solves_wall=round(wall["solves"] / args.steps, 2),
                                  grads_wall=round(wall["grads"] / args.steps, 2)),
               schedule="forward and adjoint concurrent" if args.concurrent else "forward, then adjoint",
               forward=dict(iters=f.iters, rho_rel=f.rho_rel, true_residual=true_res, ell=f.ell, status=f.status,
                            projected=f.proj),
               adjoint=dict(iters=a.iters, rho_rel=a.rho_rel, ell=a.ell, projected=a.proj))
    if not args.no_fp64_compare and args.precision == "mixed":
        one_step("fp64", profile=dominant)  # warm-up: FP64 workspaces differ from the mixed ones
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f64, a64, _ = one_step("fp64", profile=dominant)  # timed as the mixed steps are
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t1
        out["fp64_step"] = dict(ms=round(1000.0 * el64, 2), block_steps_per_s=round((f64.iters + a64.iters) / el64, 2),
                                speedup_mixed_over_fp64=round(1000.0 * el64 / ms_step, 3),
                                rho_rel=f64.rho_rel,
                                true_residual=skr.true_residual(A, B, f64.X1, f64.X2, C1, C2),
                                time_split_ms=dict(block_steps=round(f64.ms_steps + a64.ms_steps, 2),
                                                   projected_solves=round(f64.ms_proj + a64.ms_proj, 2),
                                                   recovery=round(f64.ms_recover + a64.ms_recover, 2)),
                                projected=dict(forward=f64.proj, adjoint=a64.proj))
    # Algorithm 2 (t-PKSM: the same block steps with no embedding) on the same forward
    # problem and window, for comparison with s-PKSM
    if not args.no_tpksm:
        out["tpksm_forward"] = tpksm_leg(skr, torch, A, B, C1, C2, params(args.precision, profile=True))
    if not args.no_sorth:
        out["sketched_orth_forward"] = sorth_leg(skr, torch, A, B, C1, C2, params(args.precision, profile=True), f_warm)
    if not args.no_srht:
        out["srht_forward"] = srht_leg(skr, torch, A, B, C1, C2, params(args.precision, profile=True), f_warm)
    if not args.no_lyapunov:
        out["lyapunov_forward"] = lyapunov_leg(skr, torch, A, C1, params(args.precision, profile=True), f_warm)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out))


def sorth_leg(skr, torch, A, B, C1, C2, prm, f_euc):
    """The forward solve with the truncated orthogonalisation in the sketched inner product
    (appendix A) on the same problem and window, beside the Euclidean block steps."""
    prm["orth"] = "sketched"
    skr.solve(A, B, C1, C2, **prm)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fs = skr.solve(A, B, C1, C2, **prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    return dict(ms=round(1000.0 * el, 2), block_steps_per_s=round(fs.iters / el, 1), iters=fs.iters,
                time_split_ms=dict(block_steps=round(fs.ms_steps, 2), projected_solves=round(fs.ms_proj, 2),
                                   recovery=round(fs.ms_recover, 2)),
                euclidean_forward_block_steps_ms=round(f_euc.ms_steps, 2),
                kernel_families={k: dict(launches=v[0], ms=round(v[1], 3)) for k, v in fs.kernels.items()},
                rho_rel=fs.rho_rel, true_residual=skr.true_residual(A, B, fs.X1, fs.X2, C1, C2),
                projected=fs.proj)


def srht_leg(skr, torch, A, B, C1, C2, prm, f_sparse):
    """The forward solve with the subsampled randomized DCT embedding of the paper's
    experiments (Sec. 6) instead of the sparse sign one, same problem, s and window."""
    prm["sketch"] = "srht"
    skr.solve(A, B, C1, C2, **prm)  # warm-up (also builds the sampled-row plans)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fs = skr.solve(A, B, C1, C2, **prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    fam = {k: dict(launches=v[0], ms=round(v[1], 3)) for k, v in fs.kernels.items()}
    return dict(ms=round(1000.0 * el, 2), block_steps_per_s=round(fs.iters / el, 1), iters=fs.iters,
                time_split_ms=dict(block_steps=round(fs.ms_steps, 2), projected_solves=round(fs.ms_proj, 2),
                                   recovery=round(fs.ms_recover, 2)),
                sparse_sign_forward_block_steps_ms=round(f_sparse.ms_steps, 2), kernel_families=fam,
                rho_rel=fs.rho_rel, true_residual=skr.true_residual(A, B, fs.X1, fs.X2, C1, C2),
                projected=fs.proj)


def lyapunov_leg(skr, torch, A, C1, prm, f_sylv):
    """The Lyapunov specialisation A X + X A^T = C1 C1^T on the same operator and window: one
    Krylov space instead of two (compare its block-step time with the Sylvester solve's)."""
    skr.lyap_solve(A, C1, **prm)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fl = skr.lyap_solve(A, C1, **prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    return dict(ms=round(1000.0 * el, 2), block_steps_per_s=round(fl.iters / el, 1),
                time_split_ms=dict(block_steps=round(fl.ms_steps, 2), projected_solves=round(fl.ms_proj, 2),
                                   recovery=round(fl.ms_recover, 2)),
                sylvester_forward_block_steps_ms=round(f_sylv.ms_steps, 2), rho_rel=fl.rho_rel,
                projected=fl.proj)


def tpksm_leg(skr, torch, A, B, C1, C2, prm_t):
    """Algorithm 2 (t-PKSM: the same block steps with no embedding) on the same forward
    problem and window, for comparison with s-PKSM."""
    prm_t["sketch"] = "none"
    skr.solve(A, B, C1, C2, **prm_t)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ft = skr.solve(A, B, C1, C2, **prm_t)
    torch.cuda.synchronize()
    elt = time.perf_counter() - t1
    return dict(ms=round(1000.0 * elt, 2), block_steps_per_s=round(ft.iters / elt, 1),
                time_split_ms=dict(block_steps=round(ft.ms_steps, 2), projected_solves=round(ft.ms_proj, 2),
                                   recovery=round(ft.ms_recover, 2)),
                rho_rel=ft.rho_rel, true_residual=skr.true_residual(A, B, ft.X1, ft.X2, C1, C2), projected=ft.proj)


if __name__ == "__main__":
    main()
