"""Benchmark of the sketched product C ~= A S S^T B on one MI355X.

One step = the whole path through the C ABI (os_matmul: prepare the sketch,
sketch A's columns, sketch B's rows, grouped FP32 MFMA product over the kept
blocks) on resident synthetic inputs:

    A 8192 x 32768 and B 32768 x 8192, each a rank-64 Gaussian factor product
    (shared factor) plus N(0, 0.1^2) noise, FP32; count-sketch blocks of width
    b = 1024, N = 8 needed + e = 2 extra, 2 random blocks dropped by the keep
    mask.

Reported (one JSON line): effective TFLOP/s = 2 m n l / t_step, the roofline
of the dominant kernel (the MFMA block product, timed with HIP events on its
own stream), per-stage times, the relative Frobenius error against the FP64
exact AB, the exact FP32 GEMM on the same GPU (torch.matmul) as the
comparator, and the FP64 CPU oracle timed on a bounded sample of the same
workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sketched AB eff. TFLOP/s (2mnl/t) at fixed rel-Frob err vs exact GEMM, 1 GPU"

# HBM traffic of one gemm_kept launch at the default workload, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE; KiB per
# dispatch), each scaled by what the counter reads for a plain 1 GiB device
# copy (bench.py --calibrate-copy: FETCH_SIZE 524300 KiB -> x 2.000,
# WRITE_SIZE 1048576 KiB -> x 1.000).  Commands and raw figures:
# profiles/gemm_kept_8192x8192_K8x1024_hbm_traffic.md.  Valid only for the
# kernel source it was measured on (SHA-256 of that source, see
# gemm_kept_source_sha); None otherwise.
GEMM_TRAFFIC = {
    "source_sha256": "ee137acdc8a2b26164ec93737ebf3ba4c99d9ef096488bbb2e31815ac7a6e674",
    "workload": (8192, 32768, 8192, 1024, 8, 2),
    "fetch_kib": 1573130.3, "fetch_scale": 2.000,
    "write_kib": 262144.0, "write_scale": 1.000,
}
FP32_MFMA_PEAK_TFLOPS = 157.3       # MI355X dense FP32 matrix peak
BF16_MFMA_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix peak
FP8_MFMA_PEAK_TFLOPS = 5000.0       # MI355X dense FP8 matrix peak
HBM_PEAK_GBS = 8000.0               # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--m", type=int, default=8192)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--l", type=int, default=8192)
    p.add_argument("--b", type=int, default=1024)
    p.add_argument("--N", type=int, default=8)
    p.add_argument("--e", type=int, default=2)
    p.add_argument("--drop", type=int, default=2)
    p.add_argument("--seed", type=int, default=2)
    p.add_argument("--kept-only", action="store_true")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-rows", type=int, default=6144,
                   help="rows of A and columns of B in the CPU oracle sample")
    p.add_argument("--no-layer", action="store_true",
                   help="skip the sketched linear layer (backward with a sketched weight gradient)")
    p.add_argument("--no-precision", action="store_true",
                   help="skip the BF16 / split-BF16 variants of the block product")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the batch of 64 sketched interior-point Hessians")
    p.add_argument("--no-paper", action="store_true",
                   help="skip the paper's constant-matrix workloads (Fig. 5b, Section 5.3)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain 1 GiB device copy (3 times): the reference kernel "
                        "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def gemm_kept_source_sha(path):
    """SHA-256 of the source that the FP32 gemm_kept launch compiles from:
    gemm.hip up to the FP8 kernel (helpers and gemm_kept_kernel) plus the
    launch_gemm_kept function; edits elsewhere in the file keep the counters
    valid."""
    import hashlib
    text = open(path).read()
    head = text[:text.index("// FP8 (E4M3) operands")]
    a = text.index("hipError_t launch_gemm_kept(")
    launch = text[a:text.index("\n}\n", a) + 3]
    return hashlib.sha256((head + launch).encode()).hexdigest()


def gemm_traffic_bytes(m, n, l, b, N, e):
    """Measured HBM bytes per gemm_kept launch, or None if the kernel source
    or the workload differs from the one the counters were taken on."""
    src = os.path.join(ROOT, "paper_1811_02653_amd", "csrc", "gemm.hip")
    sha = gemm_kept_source_sha(src)
    t = GEMM_TRAFFIC
    if sha != t["source_sha256"] or (m, n, l, b, N, e) != t["workload"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def event_time_ms(torch, fn, reps, stream):
    """Average duration of fn() over reps launches, HIP events on `stream`."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        fn()
        start.record(stream)
        for _ in range(reps):
            fn()
        stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def bench_hessian_batch(torch, osk, args, stream, reps):
    import synthetic
    from paper_1811_02653_amd.gram import PRODUCT, PREPARE, SKETCH
    count, N, e = 64, 6, 1
    sizes, As, ds = synthetic.hessian_batch_device(count, args.seed)
    keeps = [synthetic.random_keep(N, e, args.seed + k, drop=1) for k in range(count)]
    bs = [(m + 1) // 2 for m in sizes]
    gb = osk.GramBatch(As, ds, b=bs, N=N, e=e, keeps=keeps, seeds=list(range(count)),
                       stream=stream)
    tuned_ms = gb.autotune(reps=2, stream=stream)
    tile, grid = gb.config
    # the product alone for each tile side (the autotuner times whole runs)
    by_tile = {}
    for t in (256, 128):
        gb.configure(t, 0, stream=stream)
        by_tile[t] = event_time_ms(torch, lambda: gb.run(PRODUCT, stream=stream), reps, stream)
    gb.configure(tile, grid, stream=stream)
    g = gb.graph()                      # captured on a private stream
    t_graph = event_time_ms(torch, lambda: g.launch(stream), reps, stream)
    t_eager = event_time_ms(torch, lambda: gb.run(stream=stream), reps, stream)
    t_prep = event_time_ms(torch, lambda: gb.run(PREPARE, stream=stream), reps, stream)
    t_sketch = event_time_ms(torch, lambda: gb.run(SKETCH, stream=stream), reps, stream)
    t_prod = event_time_ms(torch, lambda: gb.run(PRODUCT, stream=stream), reps, stream)
    g.close()
    K = N                                      # one of the N+e blocks dropped per problem
    exact_flops = sum(2.0 * m * m * 20 * m for m in sizes)
    # algorithmic flops of the batched product: the upper triangle with the
    # diagonal, 2*K*b per entry
    prod_flops = sum(float(m) * (m + 1) * K * b for m, b in zip(sizes, bs))
    sketch_bytes = sum(4.0 * (m * 20 * m + 20 * m + m * K * osk.block_stride(b))
                       for m, b in zip(sizes, bs))
    # exact Hessians (FP32 hipBLASLt) for the error and the exact baseline
    errs = []
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t_exact = 0.0
    for k in range(count):
        t0.record(stream)
        W = As[k] * torch.sqrt(ds[k])[None, :]
        Hx = torch.matmul(W, W.t())
        t1.record(stream)
        t1.synchronize()
        t_exact += t0.elapsed_time(t1)
        errs.append((torch.linalg.norm(gb.H[k].double() - Hx.double()) /
                     torch.linalg.norm(Hx.double())).item())
        del W, Hx
    res = {
        "workload": "64 interior-point Hessians A_k D_k A_k^T, A_k m_k x 20m_k ~ N(0,1), "
                    "m_k uniform in [500, 4000], d_k log-uniform in [1e-6, 1e6]; "
                    "b_k = ceil(m_k/2), N=6, e=1, one block dropped per problem",
        "m_k": sizes, "input_gb": sum(4.0 * m * 20 * m for m in sizes) / 1e9,
        "tile": tile, "grid": grid, "autotune_ms": tuned_ms,
        "product_ms_by_tile": by_tile,
        "ms_per_batch": t_graph, "ms_per_batch_eager": t_eager,
        "hessians_per_s": count / (t_graph * 1e-3),
        "eff_tflops": exact_flops / (t_graph * 1e-3) / 1e12,
        "stages_ms": {"prepare": t_prep, "sketch": t_sketch, "product": t_prod},
        "product_roofline": {
            "kernel": "gemm_batch_sym (FP32 v_mfma_f32_32x32x2_f32, persistent, tile %d)" % tile,
            "bound": "mfma", "unit": "TFLOP/s", "peak": FP32_MFMA_PEAK_TFLOPS,
            "algorithmic_flops_per_launch": prod_flops,
            "achieved": prod_flops / (t_prod * 1e-3) / 1e12,
            "frac": prod_flops / (t_prod * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS},
        "sketch_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "algorithmic_bytes": sketch_bytes,
            "achieved": sketch_bytes / (t_sketch * 1e-3) / 1e9,
            "frac": sketch_bytes / (t_sketch * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "exact": {"kind": "torch.matmul FP32 of A_k D_k^{1/2} with its transpose, per problem",
                  "ms": t_exact, "tflops": exact_flops / (t_exact * 1e-3) / 1e12,
                  "speedup_of_sketched": t_exact / t_graph},
        "rel_frob_vs_exact": {"mean": float(np.mean(errs)), "max": float(np.max(errs)),
                              "min": float(np.min(errs))},
    }
    log("hessian batch: tile %d grid %d, %.3f ms per batch (graph), %.3f eager; prepare %.3f, "
        "sketch %.3f, product %.3f ms (%.1f TFLOP/s); exact %.1f ms; error mean %.3e" %
        (tile, grid, t_graph, t_eager, t_prep, t_sketch, t_prod,
         res["product_roofline"]["achieved"], t_exact, res["rel_frob_vs_exact"]["mean"]))
    gb.close()
    del gb, As, ds
    torch.cuda.empty_cache()
    return res


def _predicted_rel_frob(nA2, nB2, nAB2, cross, K, b):
    """RMS relative Frobenius error of the sketched product for K kept
    count-sketch blocks of width b: Lemma 1's variance summed over the
    entries of AB and divided by K, over |AB|_F^2."""
    return ((nA2 * nB2 + nAB2 - 2.0 * cross) / (K * b) / nAB2) ** 0.5


def bench_paper_workloads(torch, osk, args, stream, reps):
    import synthetic
    dev = "cuda"
    res = {}
    # Fig. 5b: A(x, y) = x + y, m = l = 10b, n = 60b, b = 2048, B = A^T,
    # z = 30b; e of the 30 workers of every b x b block of C ignored; the
    # paper's error is a mean over ten sketches (0.8 % at e = 4)
    b, nb = 2048, 30
    m, n = 10 * b, 60 * b
    A, x, y = synthetic.paper_matrices_device(m, n, device=dev)
    G, nA2, _, cross = synthetic.paper_exact_products(x, y)
    nG2 = torch.sum(G * G).item()
    bp = osk.block_stride(b)
    At = torch.empty((m, nb * bp), dtype=torch.float32, device=dev)
    C = torch.empty((m, m), dtype=torch.float32, device=dev)
    es, inst = (0, 2, 4, 6, 8, 10), 10
    errs = {e_: [] for e_ in es}
    t_sk, t_gemm = None, {}
    for k in range(inst):
        seed = args.seed + 100 + k
        prep = osk.sketch_prepare(n, b, nb, 0, seed=seed)
        # B = A^T: the sketch of B's rows is the sketch of A's columns
        sk = lambda: osk.sketch_cols(A, b, nb, 0, seed=seed, prep=prep, out=At, stream=stream)
        if k == 0:
            t_sk = event_time_ms(torch, sk, 3, stream)
        else:
            with torch.cuda.stream(stream):
                sk()
        for e_ in es:
            cm = torch.from_numpy(synthetic.random_cmask(m // b, m // b, nb - e_, e_,
                                                         seed * 100 + e_)).to(dev)
            g = lambda: osk.gemm_kept_cmask(At, At, b, cm, out=C, stream=stream)
            if k == 0:
                t_gemm[e_] = event_time_ms(torch, g, 2, stream)
            else:
                with torch.cuda.stream(stream):
                    g()
            stream.synchronize()
            errs[e_].append((torch.sum((C.double() - G) ** 2).item() / nG2) ** 0.5)
    res["fig5b"] = {
        "workload": "A(x,y) = x + y, m = l = 20480, n = 122880, B = A^T, b = 2048, z = 30b; e "
                    "of the 30 workers of every b x b block of C dropped at random",
        "e": list(es), "instances": inst,
        "rel_frob_mean": [float(np.mean(errs[e_])) for e_ in es],
        "rel_frob_predicted_rms": [_predicted_rel_frob(nA2, nA2, nG2, cross, nb - e_, b)
                                   for e_ in es],
        "paper_printed": {"e": 4, "rel_frob_mean": 0.008},
        "sketch_ms": t_sk,
        "gemm_cmask_ms": [t_gemm[e_] for e_ in es],
        "gemm_cmask_tflops": [2.0 * m * m * (nb - e_) * bp / (t_gemm[e_] * 1e-3) / 1e12
                              for e_ in es],
    }
    log("Fig. 5b: mean error by e %s (predicted %s); sketch %.2f ms, product %s ms" % (
        ["%.4f" % v for v in res["fig5b"]["rel_frob_mean"]],
        ["%.4f" % v for v in res["fig5b"]["rel_frob_predicted_rms"]], t_sk,
        ["%.1f" % v for v in res["fig5b"]["gemm_cmask_ms"]]))
    del A, G, At, C, x, y
    torch.cuda.empty_cache()
    # Section 5.3: A(x, y) = x + y and B(x, y) = x y, both n x n, b = 4000,
    # z = n/2 + b, one worker per block of C ignored (error under 2 %)
    b = 4000
    rows = []
    for n in (24000, 40000):
        nb = n // (2 * b) + 1
        A, B, x, y, z = synthetic.paper_matrices_device(n, n, n, device=dev)
        AB, nA2, nB2, cross = synthetic.paper_exact_products(x, y, z)
        nAB2 = torch.sum(AB * AB).item()
        ws = torch.empty(osk.workspace_bytes(n, n, n, b, nb - 1, 1), dtype=torch.uint8, device=dev)
        C = torch.empty((n, n), dtype=torch.float32, device=dev)
        errs, t = [], None
        for k in range(inst):
            seed = args.seed + n + k
            cm = torch.from_numpy(synthetic.random_cmask(n // b, n // b, nb - 1, 1, seed)).to(dev)
            f = lambda: osk.matmul_cmask(A, B, b, nb - 1, 1, cm, seed=seed, out=C, workspace=ws,
                                         stream=stream)
            if k == 0:
                t = event_time_ms(torch, f, 2, stream)
            else:
                with torch.cuda.stream(stream):
                    f()
            stream.synchronize()
            errs.append((torch.sum((C.double() - AB) ** 2).item() / nAB2) ** 0.5)
        rows.append({"n": n, "blocks": nb, "ms": t,
                     "eff_tflops": 2.0 * n ** 3 / (t * 1e-3) / 1e12,
                     "rel_frob_mean": float(np.mean(errs)),
                     "rel_frob_predicted_rms": _predicted_rel_frob(nA2, nB2, nAB2, cross,
                                                                   nb - 1, b)})
        del A, B, AB, C, ws, x, y, z
        torch.cuda.empty_cache()
    res["section_5_3"] = {
        "workload": "A(x,y) = x + y and B(x,y) = x y, n x n, b = 4000, z = n/2 + b, one of the "
                    "z/b workers of every b x b block of C dropped at random",
        "instances": inst, "paper_printed": "error under 2 %, decreasing with n", "runs": rows}
    log("Section 5.3: %s" % ", ".join("n=%d err %.4f (pred %.4f) %.1f ms" % (
        r["n"], r["rel_frob_mean"], r["rel_frob_predicted_rms"], r["ms"]) for r in rows))
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_02653_amd as osk
    import synthetic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 1 << 30,
                          "bytes_written": 1 << 30, "launches": 3}))
        return
    osk.lib()    # fails loudly when the HIP library is not built

    m, n, l, b, N, e = args.m, args.n, args.l, args.b, args.N, args.e
    dev = torch.device("cuda:0")
    t0 = time.time()
    A_h, B_h = synthetic.lowrank_pair(m, n, l, args.seed, rank=64, noise=0.1)
    keep = synthetic.random_keep(N, e, args.seed, drop=args.drop)
    log("inputs generated in %.1f s; keep mask %s" % (time.time() - t0, keep.tolist()))
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    C = torch.empty((m, l), dtype=torch.float32, device=dev)
    ws = torch.empty(osk.workspace_bytes(m, n, l, b, N, e),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        osk.matmul(A, B, b, N, e, seed=args.seed, keep=keep, kept_only=args.kept_only, out=C,
                   workspace=ws, stream=stream)

    # ---- timed region: K whole-path steps
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    eff_tflops = 2.0 * m * n * l / (ms_per_step * 1e-3) / 1e12
    log("step %.3f ms -> %.1f eff TFLOP/s" % (ms_per_step, eff_tflops))

    # ---- per-stage times (same kernels, called one stage at a time)
    bp = osk.block_stride(b)
    nst = osk.stored_count(N, e, keep, args.kept_only)
    K = int(np.count_nonzero(keep))
    prep = osk.sketch_prepare(n, b, N, e, seed=args.seed)
    At = torch.empty((m, nst * bp), dtype=torch.float32, device=dev)
    Bt = torch.empty((l, nst * bp), dtype=torch.float32, device=dev)
    stored_keep = None if args.kept_only else keep      # mask over the stored blocks
    tws = torch.empty(osk.sketch_rows_workspace_bytes(n, l), dtype=torch.uint8, device=dev)
    reps = max(3, args.steps)
    t_prep = event_time_ms(torch, lambda: osk.sketch_prepare(n, b, N, e, seed=args.seed,
                                                             stream=stream), reps, stream)
    t_sa = event_time_ms(torch, lambda: osk.sketch_cols(A, b, N, e, seed=args.seed, keep=keep,
                                                        kept_only=args.kept_only, prep=prep,
                                                        out=At, stream=stream),
                        reps, stream)
    t_sb = event_time_ms(torch, lambda: osk.sketch_rows(B, b, N, e, seed=args.seed, keep=keep,
                                                        kept_only=args.kept_only, prep=prep,
                                                        out=Bt, workspace=tws, stream=stream),
                        reps, stream)
    t_gemm = event_time_ms(torch, lambda: osk.gemm_kept(At, Bt, b, keep=stored_keep, out=C,
                                                        stream=stream), reps, stream)
    gemm_flops = 2.0 * m * l * K * bp
    gemm_tflops = gemm_flops / (t_gemm * 1e-3) / 1e12
    sketch_bytes_a = 4.0 * (m * n + m * nst * bp)
    sketch_bytes_b = 4.0 * (n * l + l * nst * bp)
    log("stages: prepare %.3f, sketch A %.3f, sketch B %.3f, gemm %.3f ms" %
        (t_prep, t_sa, t_sb, t_gemm))

    # ---- accuracy against the exact FP64 product (computed on the GPU)
    step()
    torch.cuda.synchronize()
    AB = torch.matmul(A.double(), B.double())
    Cd = C.double()
    diff2 = torch.sum((Cd - AB) ** 2).item()
    ab2 = torch.sum(AB ** 2).item()
    a2 = torch.sum(A.double() ** 2).item()
    b2 = torch.sum(B.double() ** 2).item()
    rel_err = (diff2 / ab2) ** 0.5
    norm_err2 = diff2 / (a2 * b2)
    del Cd

    # ---- speedup against error: whole steps for N in {2, 4, 8, 16} (e = 2,
    # two random blocks dropped, the same inputs), and the headline with the
    # dropped blocks skipped at sketch time
    sweep = []
    for Ns in (2, 4, 8, 16):
        ks = synthetic.random_keep(Ns, e, args.seed, drop=args.drop)
        wss = torch.empty(osk.workspace_bytes(m, n, l, b, Ns, e), dtype=torch.uint8, device=dev)
        t_s = event_time_ms(torch, lambda: osk.matmul(A, B, b, Ns, e, seed=args.seed, keep=ks,
                                                      out=C, workspace=wss, stream=stream),
                            reps, stream)
        Cd = C.double()
        sweep.append({"N": Ns, "e": e, "kept_blocks": int(np.count_nonzero(ks)), "ms": t_s,
                      "eff_tflops": 2.0 * m * n * l / (t_s * 1e-3) / 1e12,
                      "rel_frob_vs_exact_fp64": (torch.sum((Cd - AB) ** 2).item() / ab2) ** 0.5})
        del wss, Cd
    t_kept_only = event_time_ms(torch, lambda: osk.matmul(A, B, b, N, e, seed=args.seed,
                                                          keep=keep, kept_only=True, out=C,
                                                          workspace=ws, stream=stream),
                                reps, stream)
    log("N sweep: %s; kept_only step %.3f ms" %
        (", ".join("N=%d %.2f ms err %.4f" % (r["N"], r["ms"], r["rel_frob_vs_exact_fp64"])
                   for r in sweep), t_kept_only))
    del AB
    torch.cuda.empty_cache()
    step()

    # ---- exact FP32 GEMM on the same GPU: the vendor library, and the block
    # product kernel itself run on A and B^T unsketched (the inner dimension
    # split into 4 blocks of n/4, all kept: C = AB / 4 with the same flops as
    # AB)
    Cx = torch.empty((m, l), dtype=torch.float32, device=dev)
    t_exact = event_time_ms(torch, lambda: torch.matmul(A, B, out=Cx), 3, stream)
    t_exact_own = None
    if n % 4 == 0 and (n // 4) % 32 == 0 and n // 4 <= 8192:
        BT = B.t().contiguous()
        t_exact_own = event_time_ms(torch, lambda: osk.gemm_kept(A, BT, n // 4, out=Cx,
                                                                 stream=stream), 3, stream)
        del BT
    del Cx
    torch.cuda.empty_cache()

    # ---- reduced-precision block product (BF16 or FP8 operands with
    # power-of-two block scales, FP32 accumulation; split forms add residuals):
    # whole steps, the block product alone, and the error against the exact
    # FP64 AB, on the same inputs; then the same errors on inputs with
    # log-normal (sigma = 2) row norms of A and column norms of B
    precision = None
    if not args.no_precision:
        precision = {}
        AB = torch.matmul(A.double(), B.double())
        ab_norm = torch.linalg.norm(AB).item()
        C32 = C.double()
        for prec in ("bf16", "bf16x3", "fp8", "fp8x3"):
            wsp = torch.empty(osk.workspace_bytes(m, n, l, b, N, e, precision=prec),
                              dtype=torch.uint8, device=dev)
            Cp = torch.empty((m, l), dtype=torch.float32, device=dev)

            def pstep():
                osk.matmul(A, B, b, N, e, seed=args.seed, keep=keep, kept_only=args.kept_only,
                           out=Cp, workspace=wsp, stream=stream, precision=prec)

            for _ in range(args.warmup):
                pstep()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                pstep()
            torch.cuda.synchronize()
            p_ms = 1e3 * (time.perf_counter() - t0) / args.steps
            QA = osk.sketch_quantize(At, b, nst, precision=prec)
            QB = osk.sketch_quantize(Bt, b, nst, precision=prec)
            t_q = event_time_ms(torch, lambda: osk.sketch_quantize(At, b, nst, precision=prec,
                                                                    out=QA, stream=stream),
                                reps, stream)
            t_pg = event_time_ms(torch, lambda: osk.gemm_kept_prec(QA, QB, b, nst, precision=prec,
                                                                    keep=stored_keep, out=Cp,
                                                                    stream=stream),
                                 reps, stream)
            bq = osk.block_stride_prec(b, prec)
            flops = 2.0 * m * l * K * bq * (3 if prec.endswith("x3") else 1)
            peak = FP8_MFMA_PEAK_TFLOPS if prec.startswith("fp8") else BF16_MFMA_PEAK_TFLOPS
            pstep()
            torch.cuda.synchronize()
            Cd = Cp.double()
            precision[prec] = {
                "ms_per_step": p_ms,
                "eff_tflops": 2.0 * m * n * l / (p_ms * 1e-3) / 1e12,
                "gemm_ms": t_pg,
                "gemm_tflops": flops / (t_pg * 1e-3) / 1e12,
                "gemm_peak_tflops": peak,
                "gemm_frac_of_peak": flops / (t_pg * 1e-3) / 1e12 / peak,
                "quantize_ms_per_sketch": t_q,
                "rel_frob_vs_exact_fp64": (torch.linalg.norm(Cd - AB).item() / ab_norm),
                "rel_frob_vs_fp32_path": (torch.linalg.norm(Cd - C32).item() /
                                          torch.linalg.norm(C32).item()),
            }
            log("%s: step %.3f ms (%.1f eff TFLOP/s), block product %.3f ms (%.1f TFLOP/s), "
                "error vs exact %.4e" % (prec, p_ms, precision[prec]["eff_tflops"], t_pg,
                                         precision[prec]["gemm_tflops"],
                                         precision[prec]["rel_frob_vs_exact_fp64"]))
            del wsp, QA, QB, Cd
        del AB, C32
        torch.cuda.empty_cache()
        # error on log-normal row / column norms (same shapes, same sketch)
        A2_h, B2_h = synthetic.lognormal_scaled_pair(m, n, l, args.seed, sigma=2.0)
        A2 = torch.from_numpy(A2_h).to(dev)
        B2 = torch.from_numpy(B2_h).to(dev)
        del A2_h, B2_h
        AB2 = torch.matmul(A2.double(), B2.double())
        n2 = torch.linalg.norm(AB2).item()
        lognormal, vs32 = {}, {}
        C2 = None
        for prec in ("fp32", "bf16", "bf16x3", "fp8", "fp8x3"):
            Cq = osk.matmul(A2, B2, b, N, e, seed=args.seed, keep=keep, precision=prec)
            torch.cuda.synchronize()
            lognormal[prec] = torch.linalg.norm(Cq.double() - AB2).item() / n2
            if prec == "fp32":
                C2 = Cq.double()
            else:
                vs32[prec] = torch.linalg.norm(Cq.double() - C2).item() / torch.linalg.norm(C2).item()
            del Cq
        precision["lognormal_rows_cols_sigma2"] = {"rel_frob_vs_exact_fp64": lognormal,
                                                   "rel_frob_vs_fp32_path": vs32}
        del C2
        log("log-normal norms, error vs exact: %s" % lognormal)
        del A2, B2, AB2
        torch.cuda.empty_cache()

    # ---- sketched linear layer: X 16384 x 4096 and W 4096 x 4096 in BF16,
    # dY ~ N(0, 1); the weight gradient X^T dY sketched over the 16384 tokens
    # (b = 512, N = 4, e = 0) against the exact BF16 GEMM
    layer = None
    if not args.no_layer:
        from paper_1811_02653_amd.autograd import sketched_weight_grad
        T_, din, dout, lb, lN = 16384, 4096, 4096, 512, 4
        Xl_h, Wl_h, Dl_h = synthetic.linear_layer(T_, din, dout, args.seed)
        Xl = torch.from_numpy(Xl_h).to(dev).to(torch.bfloat16)
        Wl = torch.from_numpy(Wl_h).to(dev).to(torch.bfloat16)
        Dl = torch.from_numpy(Dl_h).to(dev).to(torch.bfloat16)
        del Xl_h, Wl_h, Dl_h
        t_fwd = event_time_ms(torch, lambda: torch.matmul(Xl, Wl), reps, stream)
        t_dx = event_time_ms(torch, lambda: torch.matmul(Dl, Wl.t()), reps, stream)
        t_dw_exact = event_time_ms(torch, lambda: torch.matmul(Xl.t(), Dl), reps, stream)
        res = {}
        dW_exact = torch.matmul(Xl.t().float(), Dl.float()).double()
        nrm = torch.linalg.norm(dW_exact).item()
        for prec in ("fp32", "bf16"):
            t_dw = event_time_ms(torch, lambda: sketched_weight_grad(Xl, Dl, lb, lN, 0,
                                                                      seed=args.seed,
                                                                      precision=prec,
                                                                      stream=stream),
                                 reps, stream)
            dW = sketched_weight_grad(Xl, Dl, lb, lN, 0, seed=args.seed, precision=prec)
            torch.cuda.synchronize()
            res[prec] = {"dW_ms": t_dw,
                         "rel_frob_vs_exact": torch.linalg.norm(dW.double() - dW_exact).item() / nrm,
                         "backward_ms": t_dx + t_dw}
            del dW
        layer = {"workload": "X %dx%d, W %dx%d, dY %dx%d in BF16; dW sketched over the tokens, "
                             "b=%d, N=%d, e=0" % (T_, din, din, dout, T_, dout, lb, lN),
                 "forward_ms": t_fwd, "dX_ms": t_dx, "dW_exact_bf16_ms": t_dw_exact,
                 "backward_exact_ms": t_dx + t_dw_exact, "sketched_dW": res}
        log("layer: forward %.3f ms, dX %.3f ms, exact dW %.3f ms, sketched dW %s" %
            (t_fwd, t_dx, t_dw_exact, {k: round(v["dW_ms"], 3) for k, v in res.items()}))
        del Xl, Wl, Dl, dW_exact
        torch.cuda.empty_cache()

    # ---- batch of 64 sketched interior-point Hessians H_k = A_k D_k A_k^T:
    # A_k m_k x 20 m_k, m_k uniform in [500, 4000], A_k ~ N(0,1), d_k
    # log-uniform in [1e-6, 1e6], b_k = ceil(m_k / 2), N = 6, e = 1 with one
    # block dropped; sketch with D^{1/2} fused, one persistent product launch
    # over the upper-triangle tiles of all 64, the whole batch replayed as a
    # HIP graph, tile side autotuned
    batch = None
    if not args.no_batch:
        batch = bench_hessian_batch(torch, osk, args, stream, reps)

    # ---- the paper's own constant-matrix workloads at its sizes: errors
    # against its printed figures and the second-moment formula
    paper = None
    if not args.no_paper:
        paper = bench_paper_workloads(torch, osk, args, stream, reps)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    sample_err = None
    if not args.no_cpu:
        import oracle
        r = min(args.cpu_rows, m, l)
        A_s = A_h[:r, :]
        B_s = B_h[:, :r]
        t0 = time.perf_counter()
        C_ref = oracle.sketched_matmul(A_s, B_s, b, N, e, seed=args.seed, keep=keep)
        t_cpu = time.perf_counter() - t0
        cpu_tflops = 2.0 * r * n * r / t_cpu / 1e12
        cpu = {"value": cpu_tflops, "unit": "TFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "C[:%d, :%d] of the same product (A[:%d, :] and B[:, :%d], same sketch "
                         "and mask), FP64 plain loops, %.1f s" % (r, r, r, r, t_cpu)}
        sample_err = oracle.rel_frob(C[:r, :r].cpu().numpy(), C_ref)
        log("cpu oracle sample: %.1f s, rel-Frob GPU vs oracle on the sample %.2e" %
            (t_cpu, sample_err))

    out = {
        "metric": METRIC,
        "value": eff_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sketched product A %dx%d . B %dx%d, rank-64 Gaussian factor products "
                        "+ N(0,0.1^2) noise, b=%d, N=%d, e=%d, %d random blocks dropped%s"
                        % (m, n, n, l, b, N, e, args.drop,
                           ", dropped blocks skipped at sketch time" if args.kept_only else ""),
            "m": m, "n": n, "l": l, "b": b, "N": N, "e": e, "kept_blocks": K,
            "keep_mask": keep.tolist(), "seed": args.seed, "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": "gemm_kept (FP32 v_mfma_f32_32x32x2_f32)",
            "bound": "mfma",
            "achieved": gemm_tflops,
            "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": gemm_tflops / FP32_MFMA_PEAK_TFLOPS,
            "traffic": gemm_traffic_bytes(m, n, l, b, N, e),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "algorithmic_flops_per_launch": gemm_flops,
            "avg_launch_ms": t_gemm,
        },
        "cpu_baseline": cpu,
        "stages_ms": {"prepare": t_prep, "sketch_A": t_sa, "sketch_B": t_sb, "gemm": t_gemm},
        "sketch_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "sketch_A_achieved": sketch_bytes_a / (t_sa * 1e-3) / 1e9,
            "sketch_B_achieved": sketch_bytes_b / (t_sb * 1e-3) / 1e9,
            "sketch_A_frac": sketch_bytes_a / (t_sa * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "sketch_B_frac": sketch_bytes_b / (t_sb * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "error": {"rel_frob_vs_exact_fp64": rel_err,
                  "normalised_err2": norm_err2,
                  "rel_frob_vs_oracle_sample": sample_err},
        "precision_variants": precision,
        "sketched_linear_layer": layer,
        "hessian_batch": batch,
        "exact_gemm": {"kind": "torch.matmul FP32 (hipBLASLt)", "ms": t_exact,
                       "tflops": 2.0 * m * n * l / (t_exact * 1e-3) / 1e12,
                       "speedup_of_sketched": t_exact / ms_per_step,
                       "same_kernel": None if t_exact_own is None else {
                           "kind": "gemm_kept on A and B^T unsketched (4 kept blocks of n/4)",
                           "ms": t_exact_own,
                           "tflops": 2.0 * m * n * l / (t_exact_own * 1e-3) / 1e12,
                           "speedup_of_sketched": t_exact_own / ms_per_step}},
        "speedup_vs_error": {"sweep": sweep, "kept_only_ms_per_step": t_kept_only},
        "paper_workloads": paper,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
