"""Benchmark: adaptive randomized LUPP interpolative decomposition of one
large matrix on one MI355X.

Workload (default): A = U diag(sigma) V^T, 50000 x 20000, sigma_j = j^-2,
U and V from the QR of seeded Gaussian matrices, stored in FP32; adaptive
blocked LUPP-ID with sketch block 64, relative Frobenius tolerance 1e-6,
maximum rank 2048.  One step = one whole decomposition (sketch passes,
block updates, estimates, panel factorisations, interpolation solve) with A
already resident in HBM.

Prints one JSON line: ID GFLOP/s (canonical flop count, see
paper_2310_09417_amd/flops.py) as the value, decompositions per second, the
speedup over the plain FP64 path on the same matrix, a roofline entry for the
dominant kernel (its average duration from HIP events recorded around each of
its launches during the timed steps), and the CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32_mfma": 157.3e12, "f64_mfma": 78.6e12, "bf16_mfma": 2.5e15, "fp8_mfma": 5.0e15,
        "hbm": 8.0e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_09417_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy
    of known size) from the committed counter summary, if it was taken from
    the current sources of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get("kernels", {}).get(kernel)
    if not ent:
        return None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_09417_amd", "csrc")
    for f in ent.get("sources", []):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    if h.hexdigest()[:16] != ent.get("source_hash"):
        return None
    return ent.get("hbm_bytes_per_launch")


def host_cpu() -> dict:
    """Host CPU model and core count (for the record of the CPU baseline)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def fixed_rank_matrix(workloads):
    """The fixed-rank FP64 workload: 2000 x 1000, sigma_j = 10^(-10 (j-1)/999),
    U and V from the QR of seeded Gaussian matrices."""
    A, _ = workloads.fast_decay(2000, 1000, decades=10.0, seed=101)
    return A


def bench_fixed_rank(torch, rid, workloads, calls=50):
    """The fixed-rank FP64 configuration on the GPU: randLUPP of the 2000 x 1000
    matrix at k = 100 with p = 20 estimate vectors, per call (HIP events over
    `calls` calls, A resident), through the workspace form and the form
    without a caller workspace."""
    dev = torch.device("cuda:0")
    A = torch.as_tensor(fixed_rank_matrix(workloads), dtype=torch.float64).to(dev)
    m, n, k, p = 2000, 1000, 100, 20
    cfg = rid.binding._cfg(rid.RID_F64, 1, True)
    wb = rid.rid_workspace_bytes(m, n, k + p, p, cfg)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    J = torch.zeros(k, dtype=torch.int64, device=dev)
    T = torch.zeros((k, n), dtype=torch.float64, device=dev)
    ko = torch.zeros(1, dtype=torch.int32, device=dev)
    eo = torch.zeros(1, dtype=torch.float64, device=dev)
    so = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    args = (J.data_ptr(), T.data_ptr(), n, ko.data_ptr(), eo.data_ptr(), so.data_ptr())

    def call_ws():
        rc = rid.rid_lupp_fixed_rank(A.data_ptr(), m, n, n, k, p, cfg, *args, work.data_ptr(), wb,
                                     stream)
        if rc != 0:
            raise RuntimeError(f"rid_lupp_fixed_rank -> {rc}")

    def call_na():
        rc = rid.binding.rid_lupp_fixed_rank_noalloc(A.data_ptr(), m, n, n, k, p, cfg, *args,
                                                     stream)
        if rc != 0:
            raise RuntimeError(f"rid_lupp_fixed_rank_noalloc -> {rc}")

    res = {"workload": "fixed-rank randLUPP, FP64, A 2000x1000 (10 decades), k=100, p=20"}
    F = rid.flops_id(m, n, k, k + p)
    for name, fn in (("workspace", call_ws), ("noalloc", call_na)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / calls
        res[name] = {"ms_per_call": ms, "gflops": F / (ms * 1e-3) / 1e9}
        log(f"[bench] fixed rank FP64 2000x1000 k=100 p=20 ({name}): {ms:.3f} ms per call, "
            f"{F / (ms * 1e-3) / 1e9:.0f} GFLOP/s")
    res["k"] = int(ko.item())
    res["status"] = rid.status_string(int(so.item()))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=50000)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--b", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--kmax", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--lp-steps", type=int, default=3,
                    help="timed runs of each precision form (A stored in BF16 / FP8-e4m3); "
                         "0 skips them")
    ap.add_argument("--sweep", type=int, default=1,
                    help="1: precision forms over tolerances 1e-3/1e-6/1e-9 with errors "
                         "against the original matrix and the FP64 path (0 skips it)")
    ap.add_argument("--sweep-second", type=str, default="100000x10000",
                    help="second matrix shape of the sweep (empty: main shape only)")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-kmax", type=int, default=64,
                    help="rank cap of the bounded oracle sample")
    ap.add_argument("--batched", type=int, default=1,
                    help="1: time the 4096-block batched workload (0 skips it)")
    ap.add_argument("--nblk", type=int, default=4096)
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--learned-blocks", type=int, default=65536,
                    help="training blocks per form of the learned-rank section, in chunks of "
                         "4096 (0 skips it)")
    ap.add_argument("--learned-test-blocks", type=int, default=16384,
                    help="held-out blocks of the learned-rank comparison")
    ap.add_argument("--paper-sizes", type=str, default="2048,4096,8192,16384",
                    help="n of the paper's n x n Fast Decay timing workload (empty: skip)")
    ap.add_argument("--paper-steps", type=int, default=2)
    ap.add_argument("--paper-bsweep-n", type=int, default=8192,
                    help="n at which the paper workload also runs b = 32 and 64")
    ap.add_argument("--cert-p", type=int, default=8,
                    help="vectors of the a-posteriori certificate of the fp32 ID (0 skips it)")
    ap.add_argument("--rows", type=int, default=1,
                    help="1: time the row-skeleton step (two-sided ID) on the fp32 result")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the decomposition is built and timed on a single "
              f"MI355X (--gpus {args.gpus} is not supported; multi-GPU sharding is a design "
              f"note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2310_09417_amd as rid
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m, n, b, tol, kmax, seed = args.m, args.n, args.b, args.tol, args.kmax, args.seed
    rid.library()

    t0 = time.time()
    sig = workloads.sigma_power(min(m, n), 2.0)
    A64 = workloads.svd_matrix_device(m, n, sig, seed=seed, device=dev)
    A32 = A64.to(torch.float32)
    torch.cuda.synchronize()
    log(f"[bench] generated A {m}x{n} (sigma_j = j^-2) in {time.time() - t0:.1f}s")

    stream = torch.cuda.current_stream().cuda_stream
    kcap = min(kmax, m, n)

    def make_run(A, dtype_code, a_type=None, col_scale=None, refine=False, embedding=0):
        cfg = rid.binding._cfg(dtype_code, seed, True, a_type=a_type,
                               col_scale=col_scale.data_ptr() if col_scale is not None else 0,
                               refine=refine, embedding=embedding)
        wb = rid.rid_workspace_bytes(m, n, kmax, b, cfg)
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
        J = torch.zeros(kcap, dtype=torch.int64, device=dev)
        T = torch.zeros((kcap, n), dtype=torch.float64 if dtype_code == rid.RID_F64
                        else torch.float32, device=dev)
        ko = torch.zeros(1, dtype=torch.int32, device=dev)
        eo = torch.zeros(1, dtype=torch.float64, device=dev)
        so = torch.zeros(1, dtype=torch.int32, device=dev)

        def run():
            rc = rid.rid_lupp_adaptive(A.data_ptr(), m, n, A.stride(0), b, tol, kmax, cfg,
                                       J.data_ptr(), T.data_ptr(), n, ko.data_ptr(),
                                       eo.data_ptr(), so.data_ptr(), work.data_ptr(), wb, stream)
            if rc != 0:
                raise RuntimeError(f"rid_lupp_adaptive -> {rc}")

        return run, (J, T, ko, eo, so), wb

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")

    run32, out32, wb32 = make_run(A32, rid.RID_F32)
    for i in range(args.warmup):
        run32()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    rid.rid_profile_start()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run32()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = rid.rid_profile_stop()
    ms = (t1 - t0) * 1e3 / args.steps
    k = int(out32[2].item())
    E = float(out32[3].item())
    status = int(out32[4].item())
    fro = float(torch.linalg.vector_norm(A32.double()).item())
    l_drawn = k + b if k < min(m, n) else k
    F = rid.flops_id(m, n, k, l_drawn)
    gflops = F / (ms * 1e-3) / 1e9
    log(f"[bench] fp32: {ms:.2f} ms/step, k={k}, status={rid.status_string(status)}, "
        f"E/||A||={E / fro:.3e}, {gflops:.0f} GFLOP/s")
    for name, (tms, cnt) in prof.items():
        log(f"[bench]   {name:14s} {tms / args.steps:9.3f} ms/step over {cnt // args.steps} launches")

    # dominant kernel and its roofline
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    sk_ms, sk_cnt = prof["sketch"]
    sk_avg_s = sk_ms * 1e-3 / max(sk_cnt, 1)
    sk_flops = 2.0 * b * m * n  # per launch: one block of b sketch vectors over all of A
    # The 64-vector FP32 sketch multiplies on the BF16 matrix cores through an
    # exact three-part split (six BF16 products per FP32 one); its roofline is
    # HBM, algorithmic bytes = one pass over A per launch.  The FP32-equivalent
    # rate against the FP32 MFMA peak and the BF16 rate actually issued are
    # reported beside it.
    sk_bytes = 4.0 * m * n
    roof = {
        "kernel": "k_sketch (FP32 A, 64 vectors: BF16 16x16x32 MFMA on the exact three-part split; "
                  "A and Omega's operand records staged into LDS by direct copies)",
        "dominant": dom == "sketch",
        "bound": "hbm",
        "achieved": sk_bytes / sk_avg_s / 1e9,
        "peak": PEAK["hbm"] / 1e9,
        "unit": "GB/s",
        "frac": (sk_bytes / sk_avg_s) / PEAK["hbm"],
        "traffic": traffic_from_profiles("k_sketch"),
        "avg_launch_ms": sk_avg_s * 1e3,
        "algorithmic_bytes_per_launch": sk_bytes,
        "algorithmic_flops_per_launch": sk_flops,
        "fp32_equivalent": {"achieved_TFLOPs": sk_flops / sk_avg_s / 1e12,
                            "peak_TFLOPs": PEAK["f32_mfma"] / 1e12,
                            "frac": (sk_flops / sk_avg_s) / PEAK["f32_mfma"]},
        "bf16_issued": {"flops_per_launch": 6.0 * sk_flops,
                        "achieved_TFLOPs": 6.0 * sk_flops / sk_avg_s / 1e12,
                        "frac_of_bf16_peak": 6.0 * sk_flops / sk_avg_s / PEAK["bf16_mfma"]},
    }
    breakdown = {name: {"ms_per_step": tms / args.steps, "launches_per_step": cnt // args.steps}
                 for name, (tms, cnt) in prof.items()}

    # plain FP64 path on the same matrix
    fp64 = None
    if args.fp64_steps > 0:
        run64, out64, _ = make_run(A64, rid.RID_F64)
        run64()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            run64()
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / args.fp64_steps
        k64 = int(out64[2].item())
        F64 = rid.flops_id(m, n, k64, k64 + b if k64 < min(m, n) else k64)
        fp64 = {"ms_per_step": ms64, "k": k64, "status": int(out64[4].item()),
                "err_est_rel": float(out64[3].item()) / fro,
                "gflops": F64 / (ms64 * 1e-3) / 1e9, "speedup_of_fp32": ms64 / ms}
        log(f"[bench] fp64: {ms64:.2f} ms/step, k={k64}, speedup of fp32 = {ms64 / ms:.2f}x")
        del out64, run64

    def true_resid(Avals, J, T):
        """||A(:,J^c) - A(:,J) T||_F in FP64 (measurement, outside timed regions)."""
        kk = J.numel()
        mask = torch.ones(n, dtype=torch.bool, device=dev)
        mask[J] = False
        R = Avals[:, mask].double() - Avals[:, J].double() @ T[:kk, : n - kk].double()
        return float(torch.linalg.vector_norm(R).item())

    k32 = k
    resid32 = true_resid(A32, out32[0][:k32], out32[1]) / fro
    err32_orig = true_resid(A64, out32[0][:k32], out32[1]) / float(
        torch.linalg.vector_norm(A64).item())
    log(f"[bench] fp32 true residual / ||A|| = {resid32:.3e}")

    # a-posteriori certificate of the FP32 result (the check Remark 1 ends
    # with): one pass of p sketch vectors over A and the k x (n-k) product
    cert = None
    if args.cert_p > 0:
        cfgc = rid.binding._cfg(rid.RID_F32, seed, True)
        wbc = rid.rid_certificate_workspace_bytes(m, n, args.cert_p, cfgc)
        workc = torch.empty(wbc, dtype=torch.uint8, device=dev)
        Jc = out32[0][:k32].contiguous()
        certo = torch.zeros(1, dtype=torch.float64, device=dev)

        def runc():
            rc = rid.rid_certificate(A32.data_ptr(), m, n, A32.stride(0), Jc.data_ptr(), k32,
                                     out32[1].data_ptr(), n, args.cert_p, 1 << 30, cfgc,
                                     certo.data_ptr(), workc.data_ptr(), wbc, stream)
            if rc != 0:
                raise RuntimeError(f"rid_certificate -> {rc}")

        runc()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            runc()
        e1.record()
        torch.cuda.synchronize()
        msc = e0.elapsed_time(e1) / 3
        cert = {"p": args.cert_p, "ms": msc, "cert_rel": float(certo.item()) / fro,
                "resid_rel_true": resid32, "err_est_rel": E / fro}
        log(f"[bench] certificate (p={args.cert_p}) of the fp32 ID: {msc:.3f} ms, "
            f"cert/||A|| = {cert['cert_rel']:.3e} (true {resid32:.3e})")
        del workc

    # row skeletons of A(:, J) for the two-sided ID / CUR (a second, direct
    # LUPP on the 50000 x k matrix C), and the two-sided ID's error
    two_sided = None
    if args.rows:
        cfgr = rid.binding._cfg(rid.RID_F32, seed, True)
        wbr = rid.rid_rows_workspace_bytes(m, k32, cfgr)
        workr = torch.empty(wbr, dtype=torch.uint8, device=dev)
        Jr = out32[0][:k32].contiguous()
        Ir = torch.zeros(k32, dtype=torch.int64, device=dev)
        Trr = torch.zeros((k32, m), dtype=torch.float32, device=dev)
        kor = torch.zeros(1, dtype=torch.int32, device=dev)
        sor = torch.zeros(1, dtype=torch.int32, device=dev)

        def runrows():
            rc = rid.rid_lupp_rows(A32.data_ptr(), m, n, A32.stride(0), Jr.data_ptr(), k32, cfgr,
                                   Ir.data_ptr(), Trr.data_ptr(), m, kor.data_ptr(),
                                   sor.data_ptr(), workr.data_ptr(), wbr, stream)
            if rc != 0:
                raise RuntimeError(f"rid_lupp_rows -> {rc}")

        runrows()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            runrows()
        e1.record()
        torch.cuda.synchronize()
        msr_rows = e0.elapsed_time(e1) / 3
        kr = int(kor.item())
        # W A(I, J) X in FP64 on the GPU (measurement only)
        I = Ir[:kr]
        rmask = torch.ones(m, dtype=torch.bool, device=dev)
        rmask[I] = False
        Wd = torch.zeros((m, kr), dtype=torch.float64, device=dev)
        Wd[I] = torch.eye(kr, dtype=torch.float64, device=dev)
        Wd[rmask] = Trr[:kr, : m - kr].double().t()
        cmask = torch.ones(n, dtype=torch.bool, device=dev)
        cmask[Jr] = False
        Xd = torch.zeros((kr, n), dtype=torch.float64, device=dev)
        Xd[:, Jr] = torch.eye(kr, dtype=torch.float64, device=dev)
        Xd[:, cmask] = out32[1][:kr, : n - kr].double()
        S = A32[I][:, Jr].double()
        R = A32.double() - Wd @ (S @ Xd)
        e_two = float(torch.linalg.vector_norm(R).item()) / fro
        del R, Wd, Xd, S
        torch.cuda.empty_cache()
        two_sided = {"ms": msr_rows, "k": kr, "status": rid.status_string(int(sor.item())),
                     "err_rel_two_sided": e_two, "err_rel_column_id": resid32}
        log(f"[bench] row skeletons of A(:,J) ({m}x{kr}): {msr_rows:.2f} ms, two-sided ID "
            f"error {e_two:.4e} (column ID {resid32:.4e})")
        del workr

    # FP32 path with the FP64-residual refinement step on T
    refine = None
    if args.lp_steps > 0:
        runr, outr, _ = make_run(A32, rid.RID_F32, refine=True)
        runr()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.lp_steps):
            runr()
        torch.cuda.synchronize()
        msr = (time.perf_counter() - t0) * 1e3 / args.lp_steps
        kr = int(outr[2].item())
        rr = true_resid(A32, outr[0][:kr], outr[1]) / fro
        kept_unrefined = bool(kr == k32 and torch.equal(outr[1][:kr, : n - kr],
                                                        out32[1][:k32, : n - k32]))
        # the refined T itself (refine = 2 keeps it unconditionally), for the record
        run2, out2, _ = make_run(A32, rid.RID_F32, refine=2)
        run2()
        torch.cuda.synchronize()
        r2 = true_resid(A32, out2[0][:int(out2[2].item())], out2[1]) / fro
        del run2, out2
        refine = {"ms_per_step": msr, "overhead_ms": msr - ms, "k": kr,
                  "same_skeleton": bool(torch.equal(outr[0][:kr], out32[0][:k32])),
                  "resid_rel_true": rr, "resid_rel_unrefined": resid32,
                  "resid_rel_refined_step": r2,
                  "kept": "unrefined" if kept_unrefined else "refined"}
        log(f"[bench] fp32+refine: {msr:.2f} ms/step (+{msr - ms:.2f}), resid {rr:.4e} "
            f"(unrefined {resid32:.4e}, refined step {r2:.4e}; {refine['kept']} T kept)")
        del runr, outr

    # the same FP32 decomposition drawn from the sparse sign embedding (zeta =
    # 8): same MFMA sketch kernel, Omega tiles from the sparse generator
    sparse = None
    if args.lp_steps > 0:
        runs_, outs_, _ = make_run(A32, rid.RID_F32, embedding=rid.RID_EMB_SPARSE_SIGN)
        runs_()
        torch.cuda.synchronize()
        rid.rid_profile_start()
        t0 = time.perf_counter()
        for _ in range(args.lp_steps):
            runs_()
        torch.cuda.synchronize()
        mss = (time.perf_counter() - t0) * 1e3 / args.lp_steps
        profs = rid.rid_profile_stop()
        ks = int(outs_[2].item())
        rs = true_resid(A32, outs_[0][:ks], outs_[1]) / fro
        sparse = {"ms_per_step": mss, "k": ks, "status": rid.status_string(int(outs_[4].item())),
                  "err_est_rel": float(outs_[3].item()) / fro, "resid_rel_true": rs,
                  "resid_rel_true_gaussian": resid32,
                  "omega_ms_per_step": profs["omega"][0] / args.lp_steps,
                  "omega_ms_per_step_gaussian": prof["omega"][0] / args.steps}
        log(f"[bench] fp32 sparse sign: {mss:.2f} ms/step, k={ks}, resid {rs:.4e} "
            f"(gaussian {resid32:.4e}), generator {sparse['omega_ms_per_step']:.3f} ms/step")
        del runs_, outs_

    # precision forms: A stored in BF16 / FP8-e4m3 (per-128-column power-of-two
    # scale), sketch on matrix cores with FP32 accumulation, FP32 factorisation
    precision = {}
    if args.lp_steps > 0:
        for fmt, code, es in (("bf16", rid.RID_BF16, 2), ("fp8", rid.RID_FP8_E4M3, 1)):
            Aq, scale = workloads.quantize_device(A32, fmt)
            Avals = (Aq.float() if fmt == "bf16" else
                     Aq.float() * scale.repeat_interleave(128)[:n][None, :])
            froq = float(torch.linalg.vector_norm(Avals.double()).item())
            runq, outq, _ = make_run(Aq, rid.RID_F32, a_type=code, col_scale=scale)
            runq()
            torch.cuda.synchronize()
            rid.rid_profile_start()
            t0 = time.perf_counter()
            for _ in range(args.lp_steps):
                runq()
            torch.cuda.synchronize()
            msq = (time.perf_counter() - t0) * 1e3 / args.lp_steps
            profq = rid.rid_profile_stop()
            kq = int(outq[2].item())
            # after the first block (64 vectors with the norm pass) the form
            # sketches two blocks per pass over A (k_sketch_lpw): the
            # dominant launches, reported here
            pairq = profq.get("sketch_pair", (0.0, 0))[1] > 0
            skq, skc = profq["sketch_pair" if pairq else "sketch"]
            sk_avg = skq * 1e-3 / max(skc, 1)
            wq = 2 * b if pairq else b  # sketch vectors per launch
            bytes_l = float(es) * m * n
            Fq = rid.flops_id(m, n, kq, kq + b if kq < min(m, n) else kq)
            rq = true_resid(Avals, outq[0][:kq], outq[1]) / froq
            eq = true_resid(A64, outq[0][:kq], outq[1]) / float(torch.linalg.vector_norm(A64).item())
            peak_mfma = PEAK["bf16_mfma"] if fmt == "bf16" else PEAK["fp8_mfma"]
            precision[fmt] = {
                "ms_per_step": msq, "gflops": Fq / (msq * 1e-3) / 1e9, "k": kq,
                "status": rid.status_string(int(outq[4].item())),
                "err_est_rel": float(outq[3].item()) / froq,
                "resid_rel_stored": rq, "err_rel_vs_original": eq,
                "rounding_floor_rel": (2.0 ** -9 if fmt == "bf16" else 2.0 ** -4) / 3 ** 0.5,
                "speedup_vs_fp32": ms / msq,
                "speedup_vs_fp64": (fp64["ms_per_step"] / msq) if fp64 else None,
                "sketch": {"kernel": ("k_sketch_lpw (two 64-vector blocks per pass)" if pairq
                                      else "k_sketch_lpr (one 64-vector block per pass)"),
                           "vectors_per_launch": wq,
                           "avg_launch_ms": sk_avg * 1e3, "launches_per_step": skc // args.lp_steps,
                           "bound": "hbm", "algorithmic_bytes_per_launch": bytes_l,
                           "traffic": traffic_from_profiles(
                               f"k_sketch_lpw_{fmt}" if pairq else f"k_sketch_lp_{fmt}"),
                           "achieved_GBps": bytes_l / sk_avg / 1e9,
                           "frac_hbm": bytes_l / sk_avg / PEAK["hbm"],
                           "achieved_TFLOPs": 2.0 * wq * m * n / sk_avg / 1e12,
                           "frac_mfma": 2.0 * wq * m * n / sk_avg / peak_mfma},
                "kernel_breakdown": {nm: {"ms_per_step": t / args.lp_steps,
                                          "launches_per_step": c // args.lp_steps}
                                     for nm, (t, c) in profq.items()},
            }
            log(f"[bench] {fmt}: {msq:.2f} ms/step, k={kq}, "
                f"{precision[fmt]['status']}, resid={rq:.3e} (vs original A {eq:.3e}), "
                f"sketch {sk_avg * 1e3:.3f} ms per {wq}-vector launch = {bytes_l / sk_avg / 1e9:.0f} GB/s, "
                f"speedup vs fp32 {ms / msq:.2f}x")
            del Aq, scale, Avals, runq, outq

    # CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.skip_cpu:
        import oracle
        oracle.build()
        Ah = A32.double().cpu().numpy()
        t0 = time.perf_counter()
        o = oracle.rid_adaptive(Ah, b, tol, args.cpu_kmax, seed=seed)
        tc = time.perf_counter() - t0
        lc = o.k + b
        Fc = rid.flops_id(m, n, o.k, lc)
        cpu = {"value": Fc / tc / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"oracle adaptive LUPP-ID of the same {m}x{n} matrix capped at "
                         f"kmax={args.cpu_kmax} ({lc} sketch vectors, k={o.k}), {tc:.1f} s"}
        log(f"[bench] cpu oracle sample: {tc:.1f}s, {cpu['value']:.2f} GFLOP/s on "
            f"{cpu['cores']} threads")
        del Ah
        cpu["host"] = host_cpu()
        # the fixed-rank FP64 configuration (2000 x 1000, k = 100, p = 20) on
        # one host core and on all of them
        A0 = fixed_rank_matrix(workloads)
        F0 = rid.flops_id(2000, 1000, 100, 120)
        for thr in (1, 0):
            oracle.set_num_threads(thr)
            ts = []
            for _ in range(5):
                t0 = time.perf_counter()
                oracle.rid_fixed_rank(A0, 100, 20, seed=1)
                ts.append(time.perf_counter() - t0)
            key = "fixed_rank_2000x1000_one_core" if thr == 1 else "fixed_rank_2000x1000_all_cores"
            cpu[key] = {"ms_mean": 1e3 * sum(ts) / len(ts), "ms_median": 1e3 * sorted(ts)[2],
                        "threads": oracle.num_threads(),
                        "gflops": F0 / (sorted(ts)[2]) / 1e9}
            log(f"[bench] cpu oracle fixed rank 2000x1000 k=100 p=20 on {oracle.num_threads()} "
                f"thread(s): median {1e3 * sorted(ts)[2]:.1f} ms")
        oracle.set_num_threads(0)

    fixed0 = bench_fixed_rank(torch, rid, workloads)

    batched = None
    if args.batched:
        batched = bench_batched(args, torch, rid, workloads)

    learned = None
    if args.learned_blocks > 0:
        learned = bench_learned(args, torch, rid, workloads)
    paper = None
    if args.paper_sizes:
        paper = bench_paper(args, torch, rid, workloads)

    sweep = None
    if args.sweep:
        sweep = bench_precision_sweep(args, torch, rid, workloads, A64)

    rec = {
        "metric": "ID GFLOP/s + blocks/s at tol 1e-6; speedup vs plain FP64 GPU path",
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"adaptive LUPP-ID, A {m}x{n} fp32 (U diag(j^-2) V^T), "
                               f"b={b}, tol={tol:g} relative, kmax={kmax}",
                   "m": m, "n": n, "b": b, "tol": tol, "kmax": kmax, "seed": seed},
        "blocks_per_s": 1e3 / ms,
        "k": k,
        "status": rid.status_string(status),
        "err_est_rel": E / fro,
        "flops_per_step": F,
        "speedup_vs_fp64": (fp64["speedup_of_fp32"] if fp64 else None),
        "resid_rel_true": resid32,
        "err_rel_vs_fp64_matrix": err32_orig,
        "precision_forms": precision,
        "refine": refine,
        "certificate": cert,
        "sparse_sign": sparse,
        "two_sided": two_sided,
        "fp64_path": fp64,
        "kernel_breakdown": breakdown,
        "roofline": roof,
        "cpu_baseline": cpu,
        "fixed_rank_fp64": fixed0,
        "batched": batched,
        "learned_rank": learned,
        "paper_workload": paper,
        "precision_sweep": sweep,
        "source_hash": source_hash(),
    }
    torch.cuda.synchronize()
    rid.binding.rid_release()
    print(json.dumps(rec), flush=True)


def id_error_stats(torch, Aref, J, T, n, ref=None, chunk=2048):
    """Error of the ID A(:,J) [I T] P (FP64, chunked over columns; a
    measurement outside timed regions) against Aref: relative Frobenius error
    and max-abs error (absolute and relative to max|Aref|).  ref = (Jr, Tr):
    also the relative Frobenius and max-abs gap between this ID's
    reconstruction and that one's."""
    dev = Aref.device

    def recon(Jx, Tx, cols):
        # columns `cols` (ascending) of A(:,J) X, X with identity at J and T elsewhere
        kk = Jx.numel()
        pos = torch.full((n,), -1, dtype=torch.int64, device=dev)
        mask = torch.ones(n, dtype=torch.bool, device=dev)
        mask[Jx] = False
        rest = torch.nonzero(mask).squeeze(1)
        pos[rest] = torch.arange(rest.numel(), device=dev)
        X = torch.zeros((kk, cols.numel()), dtype=torch.float64, device=dev)
        pr = pos[cols]
        nz = pr >= 0
        X[:, nz] = Tx[:kk, pr[nz]].double()
        sk = torch.full((n,), -1, dtype=torch.int64, device=dev)
        sk[Jx] = torch.arange(kk, device=dev)
        ps = sk[cols]
        X[ps[~nz], torch.nonzero(~nz).squeeze(1)] = 1.0
        return Aref[:, Jx].double() @ X

    ss = ss_gap = 0.0
    mx = mx_gap = 0.0
    fro2 = 0.0
    amax = 0.0
    for c0 in range(0, n, chunk):
        cols = torch.arange(c0, min(n, c0 + chunk), device=dev)
        Ac = Aref[:, cols].double()
        fro2 += float((Ac * Ac).sum())
        amax = max(amax, float(Ac.abs().max()))
        Rc = recon(J, T, cols)
        D = Ac - Rc
        ss += float((D * D).sum())
        mx = max(mx, float(D.abs().max()))
        if ref is not None:
            G = Rc - recon(ref[0], ref[1], cols)
            ss_gap += float((G * G).sum())
            mx_gap = max(mx_gap, float(G.abs().max()))
        del Ac, Rc, D
    out = {"rel_fro": (ss / fro2) ** 0.5, "max_abs": mx, "max_abs_rel": mx / amax}
    if ref is not None:
        out["gap_rel_fro"] = (ss_gap / fro2) ** 0.5
        out["gap_max_abs"] = mx_gap
    return out


def bench_precision_sweep(args, torch, rid, workloads, A64_main):
    """The precision forms over tolerances 1e-3, 1e-6, 1e-9 on the main
    matrix shape and on a 100000 x 10000 matrix of the same spectrum: A
    stored in BF16 / FP8-e4m3 (per-128-column power-of-two scale), FP32
    factorisation with one FP64 refinement step on T, and the plain FP64 path
    at each tolerance.  Each result states its status, rank, estimate, time,
    and its relative Frobenius and max-abs error against the original FP64
    matrix and against the FP64 path's ID at the same tolerance (the FP64
    path is the one whose skeletons the parity tests hold to the oracle)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    b, kmax = args.b, args.kmax
    out = []
    shapes = [(args.m, args.n)]
    if args.sweep_second:
        shapes.append(tuple(int(x) for x in args.sweep_second.split("x")))
    for m, n in shapes:
        if (m, n) == (args.m, args.n):
            A64 = A64_main
        else:
            t0 = time.time()
            A64 = workloads.svd_matrix_device(m, n, workloads.sigma_power(min(m, n), 2.0),
                                              seed=args.seed + 7, device=dev)
            torch.cuda.synchronize()
            log(f"[bench] sweep: generated A {m}x{n} (sigma_j = j^-2) in {time.time() - t0:.1f}s")
        kcap = min(kmax, m, n)
        A32 = A64.to(torch.float32)
        forms = [("fp64", A64, rid.RID_F64, None, None, 0)]
        for fmt, code in (("bf16", rid.RID_BF16), ("fp8", rid.RID_FP8_E4M3)):
            Aq, sc = workloads.quantize_device(A32, fmt)
            if fmt == "fp8":
                Aq = Aq.view(torch.uint8)
            forms.append((fmt, Aq, rid.RID_F32, code, sc, 1))
        del A32
        for tol in (1e-3, 1e-6, 1e-9):
            ref = None
            for name, Ax, dt, at, sc, refine in forms:
                cfg = rid.binding._cfg(dt, args.seed, True, a_type=at,
                                       col_scale=sc.data_ptr() if sc is not None else 0,
                                       refine=refine)
                wb = rid.rid_workspace_bytes(m, n, kmax, b, cfg)
                work = torch.empty(wb, dtype=torch.uint8, device=dev)
                J = torch.zeros(kcap, dtype=torch.int64, device=dev)
                T = torch.zeros((kcap, n), dtype=torch.float64 if dt == rid.RID_F64
                                else torch.float32, device=dev)
                ko = torch.zeros(1, dtype=torch.int32, device=dev)
                eo = torch.zeros(1, dtype=torch.float64, device=dev)
                so = torch.zeros(1, dtype=torch.int32, device=dev)

                def call():
                    rc = rid.rid_lupp_adaptive(Ax.data_ptr(), m, n, Ax.stride(0), b, tol, kmax, cfg,
                                               J.data_ptr(), T.data_ptr(), n, ko.data_ptr(),
                                               eo.data_ptr(), so.data_ptr(), work.data_ptr(), wb,
                                               stream)
                    if rc != 0:
                        raise RuntimeError(f"rid_lupp_adaptive -> {rc}")

                call()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                call()
                e1.record()
                torch.cuda.synchronize()
                kk = int(ko.item())
                Jk = J[:kk].clone()
                errs = id_error_stats(torch, A64, Jk, T, n, ref=ref)
                if name == "fp64":
                    ref = (Jk, T.clone())
                res = {"shape": f"{m}x{n}", "form": name, "tol": tol, "k": kk,
                       "status": rid.status_string(int(so.item())),
                       "err_est_rel": float(eo.item()), "ms": float(e0.elapsed_time(e1)),
                       "refine": refine, "vs_original_fp64": errs}
                if name == "fp64":
                    res["vs_original_fp64"].pop("gap_rel_fro", None)
                out.append(res)
                log(f"[bench] sweep {m}x{n} {name:4s} tol={tol:g}: k={kk} {res['status']}, "
                    f"{res['ms']:.2f} ms, rel err {errs['rel_fro']:.3e}, max-abs {errs['max_abs']:.3e}"
                    + (f", gap to fp64 ID {errs['gap_rel_fro']:.3e} (max-abs "
                       f"{errs['gap_max_abs']:.3e})" if 'gap_rel_fro' in errs else ""))
                del work, T, J
        del forms
        if A64 is not A64_main:
            del A64
        torch.cuda.empty_cache()
    return out


def bench_paper(args, torch, rid, workloads):
    """The paper's own timing workload (Sec. 5.2, timing figures): n x n Fast
    Decay (sigma_i = 1e-16^((i-1)/(n-1)), Haar factors), FP64, absolute
    tolerances 1e-8 and 1e-4 (numerical rank about n/2 and n/4), block size
    128; plus block sizes 32 and 64 at n = 8192 and tolerance 1e-8.  Each
    configuration: one untimed run, then paper_steps timed runs (HIP events
    around the library call, workspace allocated beforehand)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    sizes = [int(x) for x in args.paper_sizes.split(",") if x]
    runs, gemms = [], []
    for n in sizes:
        t0 = time.time()
        sig = workloads.sigma_geometric(n, 16.0)
        A = workloads.svd_matrix_device(n, n, sig, seed=args.seed + n, device=dev)
        torch.cuda.synchronize()
        log(f"[bench] paper workload: generated {n}x{n} Fast Decay in {time.time() - t0:.1f}s")
        # (b, tol, stopping estimate): the Schur estimate of Alg. 1, and at
        # the b-sweep size also the Remark-1 sample and normUest estimates
        # (8 set-aside vectors)
        cases = [(128, 1e-8, 0), (128, 1e-4, 0)]
        if n == args.paper_bsweep_n:
            cases += [(32, 1e-8, 0), (64, 1e-8, 0), (128, 1e-8, 1), (128, 1e-8, 2)]
        for b, tol, est in cases:
            est3 = torch.zeros(3, dtype=torch.float64, device=dev)
            cfg = rid.binding._cfg(rid.RID_F64, args.seed, False, estimator=est,
                                   resid_p=8 if est else 0, est_out=est3.data_ptr() if est else 0)
            wb = rid.rid_workspace_bytes(n, n, n, b, cfg)
            work = torch.empty(wb, dtype=torch.uint8, device=dev)
            J = torch.zeros(n, dtype=torch.int64, device=dev)
            T = torch.zeros((n, n), dtype=torch.float64, device=dev)
            ko = torch.zeros(1, dtype=torch.int32, device=dev)
            eo = torch.zeros(1, dtype=torch.float64, device=dev)
            so = torch.zeros(1, dtype=torch.int32, device=dev)

            def run():
                rc = rid.rid_lupp_adaptive(A.data_ptr(), n, n, n, b, tol, n, cfg, J.data_ptr(),
                                           T.data_ptr(), n, ko.data_ptr(), eo.data_ptr(),
                                           so.data_ptr(), work.data_ptr(), wb, stream)
                if rc != 0:
                    raise RuntimeError(f"rid_lupp_adaptive -> {rc}")

            run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.paper_steps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.paper_steps
            k, E, st = int(ko.item()), float(eo.item()), int(so.item())
            F = rid.flops_id(n, n, k, k + b if k < n else k)
            r = {"n": n, "b": b, "tol": tol, "estimator": est, "ms": ms, "k": k,
                 "status": rid.status_string(st), "err_est": E, "gflops": F / (ms * 1e-3) / 1e9}
            if est:
                r["est3"] = [float(x) for x in est3.cpu()]
            if n == args.paper_bsweep_n and 0 < k < n:
                # true ID error (FP64 product on the GPU, outside the timing)
                mask = torch.ones(n, dtype=torch.bool, device=dev)
                mask[J[:k]] = False
                R = A[:, mask] - A[:, J[:k]] @ T[:k, : n - k]
                r["resid_true"] = float(torch.linalg.vector_norm(R).item())
                del R, mask
            log(f"[bench] paper workload n={n} b={b} tol={tol:g} est={est}: {ms:.2f} ms, k={k}, "
                f"{r['status']}, E={E:.2e}, {r['gflops']:.0f} GFLOP/s")
            if b == 128 and est == 0 and 0 < k < n:
                # the paper's non-adaptive comparison: randLUPP at the rank
                # the adaptive run found (one block of k vectors, no estimate)
                cfgf = rid.binding._cfg(rid.RID_F64, args.seed, False)
                wbf = rid.rid_workspace_bytes(n, n, k, 0, cfgf)
                workf = torch.empty(wbf, dtype=torch.uint8, device=dev)

                def runf():
                    rc = rid.rid_lupp_fixed_rank(A.data_ptr(), n, n, n, k, 0, cfgf, J.data_ptr(),
                                                 T.data_ptr(), n, ko.data_ptr(), eo.data_ptr(),
                                                 so.data_ptr(), workf.data_ptr(), wbf, stream)
                    if rc != 0:
                        raise RuntimeError(f"rid_lupp_fixed_rank -> {rc}")

                runf()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.paper_steps):
                    runf()
                e1.record()
                torch.cuda.synchronize()
                r["fixed_rank_ms"] = e0.elapsed_time(e1) / args.paper_steps
                log(f"[bench]   randLUPP at k={k} (non-adaptive): {r['fixed_rank_ms']:.2f} ms "
                    f"(adaptive / fixed {ms / r['fixed_rank_ms']:.2f})")
                del workf
            if b == 128:
                # time split over kernel classes, from one more (untimed) call
                rid.rid_profile_start()
                run()
                torch.cuda.synchronize()
                prof = rid.rid_profile_stop()
                tot = sum(v[0] for v in prof.values()) or 1.0
                r["split_ms"] = {c: round(v[0], 4) for c, v in prof.items() if v[1]}
                log("[bench]   split: " + ", ".join(
                    f"{c} {100 * v[0] / tot:.0f}%" for c, v in
                    sorted(prof.items(), key=lambda kv: -kv[1][0]) if v[0] > 0.01 * tot))
            runs.append(r)
            del work, J, T
        # context line of the paper's timing figure: one n x n FP64 GEMM (library)
        B = torch.empty_like(A)
        torch.matmul(A, A, out=B)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.paper_steps):
            torch.matmul(A, A, out=B)
        e1.record()
        torch.cuda.synchronize()
        gemm_ms = e0.elapsed_time(e1) / args.paper_steps
        gemms.append({"n": n, "ms": gemm_ms, "tflops": 2.0 * n ** 3 / (gemm_ms * 1e-3) / 1e12})
        log(f"[bench] paper workload n={n}: n x n FP64 GEMM (library) {gemm_ms:.2f} ms")
        del A, B
        torch.cuda.empty_cache()
    return {"workload": "n x n Fast Decay (16 decades), FP64, absolute tolerance, the paper's "
                        "timing experiment", "runs": runs, "gemm_fp64": gemms}


def bench_learned(args, torch, rid, workloads):
    """Learned rank on the batched workload: the rank MLP is trained on the
    GPU with labels that the batched path itself produces on generated
    kernel blocks (64-1024 per side; FP64 at 1e-8 and FP32 storage at 1e-6,
    the tolerance a feature; labels at block size 4 so that a hint can be
    finer than b = 32), its hint margin is chosen on a validation set, and
    on 16384 held-out blocks the batched call with hints (probe features and
    MLP in the same HIP graph) is compared with the plain adaptive batched
    call at b = 32."""
    import numpy as np
    from paper_2310_09417_amd import learned_rank as lr
    dev = torch.device("cuda:0")
    b, seed, chunk = 32, 100, 4096
    b_label = 4  # labels at a fine rank granularity, so hints can undercut b
    n_chunks = max(1, args.learned_blocks // chunk)
    forms = ((1e-8, torch.float64, None), (1e-6, torch.float32, torch.float64))
    t0 = time.time()
    F, k = lr.training_set(
        lambda i: workloads.kernel_blocks_device(chunk, 1000 + i, device=dev)[0], n_chunks,
        forms, b_label, seed)
    torch.cuda.synchronize()
    t1 = time.time()
    model, hist = lr.fit(F, k, epochs=30, batch=1024, seed=0)
    torch.cuda.synchronize()
    t2 = time.time()
    log(f"[bench] learned rank: {len(k)} labelled blocks ({n_chunks} x {chunk} per form) in "
        f"{t1 - t0:.1f}s, trained in {t2 - t1:.1f}s, pinball loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    del F
    val, _ = workloads.kernel_blocks_device(4096, 555, device=dev)
    test, shapes = workloads.kernel_blocks_device(args.learned_test_blocks, 77, device=dev)
    cost = np.array([m * n for (m, n, _, _) in shapes])
    order = list(np.argsort(-cost, kind="stable"))
    out = {"workload": f"{args.learned_test_blocks} held-out kernel blocks 1/|x-y|, m,n uniform "
                       f"in [64,1024], b={b}; hints from the rank MLP vs the plain adaptive "
                       f"batched call, both in HIP graphs, largest blocks first",
           "train_blocks": int(len(k)), "train_blocks_per_form": n_chunks * chunk,
           "label_and_feature_s": t1 - t0, "train_s": t2 - t1,
           "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1], "forms": {}}
    for tol, storage, factor in forms:
        name = "fp64_tol1e-8" if storage == torch.float64 else "fp32_storage_fp64_factor_tol1e-6"
        vb = val if storage == torch.float64 else [a.to(storage) for a in val]
        tb = test if storage == torch.float64 else [a.to(storage) for a in test]
        margin = lr.choose_margin(vb, model, b, tol, seed, factor=factor)
        res = lr.evaluate(tb, model, b, tol, seed, margin=margin, factor=factor, order=order,
                          graph=True, reps=3)
        a, l = res["adaptive"], res["learned"]
        ok_a = bool(np.all(a["status"] == rid.RID_OK))
        ok_l = bool(np.all(l["status"] == rid.RID_OK))
        r = {"margin": margin,
             "adaptive": {"ms": a["ms"], "blocks_per_s": len(tb) / (a["ms"] * 1e-3),
                          "mean_passes": float(a["passes"].mean()),
                          "mean_k": float(a["k"].mean()), "all_ok": ok_a},
             "learned": {"ms": l["ms"], "predict_ms": l["predict_ms"],
                         "blocks_per_s": len(tb) / (l["ms"] * 1e-3),
                         "mean_passes": float(l["passes"].mean()),
                         "mean_k": float(l["k"].mean()), "fallback": l["fallback"],
                         "fallback_rate": l["fallback"] / len(tb), "all_ok": ok_l},
             "speedup": a["ms"] / l["ms"]}
        out["forms"][name] = r
        log(f"[bench] learned rank {name} (margin {margin}): adaptive {a['ms']:.2f} ms "
            f"({r['adaptive']['mean_passes']:.2f} passes, mean k {r['adaptive']['mean_k']:.1f}), "
            f"learned {l['ms']:.2f} ms incl. {l['predict_ms']:.2f} ms features and MLP "
            f"({r['learned']['mean_passes']:.2f} passes, mean k {r['learned']['mean_k']:.1f}, "
            f"fallback {l['fallback']}/{len(tb)}), speedup {r['speedup']:.2f}x")
        del vb, tb
    # the plain FP64 path at the same tolerance as the FP32-storage form
    p64 = lr.evaluate(test, None, b, 1e-6, seed, order=order, graph=True, reps=3)["adaptive"]
    out["fp64_plain_tol1e-6_ms"] = p64["ms"]
    out["speedup_fp32_storage_learned_vs_fp64_plain_tol1e-6"] = (
        p64["ms"] / out["forms"]["fp32_storage_fp64_factor_tol1e-6"]["learned"]["ms"])
    log(f"[bench] learned rank: plain FP64 at 1e-6 {p64['ms']:.2f} ms; FP32-storage learned form "
        f"{out['speedup_fp32_storage_learned_vs_fp64_plain_tol1e-6']:.2f}x faster")
    del val, test
    torch.cuda.empty_cache()
    return out


def bench_batched(args, torch, rid, workloads):
    """The batched workload: 4096 kernel blocks 1/|x-y| with m, n uniform in
    [64, 1024], b = 32, one persistent launch captured in a HIP graph and
    replayed (largest blocks first).  Forms: the plain FP64 path at 1e-8 and
    at 1e-6, and FP32-stored blocks (half the bytes) factored in FP64 at 1e-6
    (the FP32 storage floor, about 3.4e-8 relative, lies above 1e-8)."""
    import numpy as np
    dev = torch.device("cuda:0")
    t0 = time.time()
    blocks64, shapes = workloads.kernel_blocks_device(args.nblk, 7, device=dev)
    blocks32 = [a.to(torch.float32) for a in blocks64]
    torch.cuda.synchronize()
    log(f"[bench] batched: {args.nblk} kernel blocks generated in {time.time() - t0:.1f}s")
    cost = np.array([m * n for (m, n, _, _) in shapes], dtype=np.float64)
    order = list(np.argsort(-cost, kind="stable"))
    b, seed = 32, 7

    def run(blocks, tol, factor, steps):
        plan = rid.BatchPlan(blocks, b, tol, seed=seed, order=order, factor=factor)
        # the persistent grid picked by the autotuner on this batch
        shape, shape_ms = plan.autotune()
        plan.launch()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.launch(stream=torch.cuda.current_stream().cuda_stream)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out = plan.result()
        del g, plan
        F = sum(rid.flops_id(m, n, int(k), int(k) + b if int(k) < min(m, n) else int(k))
                for (m, n, _, _), k in zip(shapes, out.k))
        st = {rid.status_string(int(v)): int((out.status == v).sum())
              for v in np.unique(out.status)}
        return ms, out, {"ms_per_batch": ms, "blocks_per_s": args.nblk / (ms * 1e-3),
                         "persistent_grid": shape,
                         "autotune_ms": {"all_cu": shape_ms[0], "three_quarters": shape_ms[1],
                                         "half": shape_ms[2]},
                         "id_gflops": F / (ms * 1e-3) / 1e9, "mean_rank": float(np.mean(out.k)),
                         "mean_passes": float(np.mean(out.passes)), "status_counts": st}

    forms = {}
    for name, blocks, tol, factor in (("fp64_tol1e-8", blocks64, 1e-8, None),
                                      ("fp64_tol1e-6", blocks64, 1e-6, None),
                                      ("fp32_storage_fp64_factor_tol1e-6", blocks32, 1e-6,
                                       torch.float64)):
        ms, out, res = run(blocks, tol, factor, args.batched_steps)
        forms[name] = res
        log(f"[bench] batched {name}: {ms:.2f} ms ({res['blocks_per_s']:.0f} blocks/s, "
            f"{res['id_gflops']:.0f} GFLOP/s, mean k {res['mean_rank']:.1f}, passes "
            f"{res['mean_passes']:.2f}; grid {res['persistent_grid']} workgroups, autotune "
            f"{res['autotune_ms']})")
        del out
    fp64_ms = forms["fp64_tol1e-6"]["ms_per_batch"]
    f32 = forms["fp32_storage_fp64_factor_tol1e-6"]
    return {
        "workload": f"{args.nblk} kernel blocks 1/|x-y| (cube separation 3-6), m,n uniform in "
                    f"[64,1024], b={b}, relative tolerance, one persistent launch in a HIP "
                    f"graph, largest blocks first",
        "a_bytes_fp64": float(8 * cost.sum()),
        "forms": forms,
        "blocks_per_s": f32["blocks_per_s"],
        "speedup_vs_fp64_same_tol": fp64_ms / f32["ms_per_batch"],
    }


if __name__ == "__main__":
    main()
