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
    "source_sha256": "6a10c4acaf956f66ea225353cd644efcda475cd34f91d105ce8c6fb012c89d70",
    "workload": (8192, 32768, 8192, 1024, 8, 2),
    "fetch_kib": 1573089.0, "fetch_scale": 2.000,
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
    p.add_argument("--no-ceilings", action="store_true",
                   help="skip the measured-ceiling kernels")
    p.add_argument("--no-small", action="store_true",
                   help="skip the small validation case and its log-normal precision sweep")
    p.add_argument("--no-stress", action="store_true",
                   help="skip the independent-factor stress case")
    p.add_argument("--profile-stage", choices=["step", "sketch_A", "sketch_B", "gemm", "prepare",
                                               "gemm_bf16", "gemm_fp8", "lib_bf16", "lib_fp8"],
                   help="run only this stage of the headline workload --steps times (after "
                        "--warmup), print nothing else: for rocprofv3 counter passes")
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
    import re
    text = open(path).read()
    head = text[:text.index("// FP8 (E4M3) operands")]
    a = text.index("hipError_t launch_gemm_kept(")
    launch = text[a:text.index("\n}\n", a) + 3]
    # comments and blank lines do not change the kernel
    code = re.sub(r"//[^\n]*", "", head + launch)
    code = "\n".join(line.rstrip() for line in code.splitlines() if line.strip())
    return hashlib.sha256(code.encode()).hexdigest()


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


def _ceilings_lib():
    import ctypes
    path = os.path.join(ROOT, "paper_1811_02653_amd", "libosk_ceilings.so")
    if not os.path.exists(path):
        raise RuntimeError("libosk_ceilings.so is not built (python -m paper_1811_02653_amd.build)")
    L = ctypes.CDLL(path)
    i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    L.osk_ceiling_copy.argtypes = [vp, vp, i64, ci, vp]
    L.osk_ceiling_read.argtypes = [vp, i64, vp, ci, vp]
    L.osk_ceiling_mfma.argtypes = [ci, ci, ci, vp, vp]
    L.osk_ceiling_lds_gather.argtypes = [ci, ci, ci, vp, vp]
    for f in (L.osk_ceiling_copy, L.osk_ceiling_read, L.osk_ceiling_mfma,
              L.osk_ceiling_lds_gather):
        f.restype = ci
    return L


def bench_ceilings(torch, stream):
    """Measured ceilings on this GPU (own HIP kernels, csrc/ceilings.hip):
    HBM copy and read-only streaming, FP32 / BF16 / FP8 MFMA loops, and
    16-byte LDS gathers at random and conflict-free addresses."""
    import ctypes
    L = _ceilings_lib()
    dev = torch.device("cuda:0")
    st = ctypes.c_void_p(stream.cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())

    def run(rc):
        if rc != 0:
            raise RuntimeError("ceiling kernel launch failed: hipError_t %d" % rc)

    out = {}
    n4 = 1 << 26                                    # 1 GiB of 16-byte elements
    src = torch.ones(4 * n4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    grid = 256 * 64
    t = event_time_ms(torch, lambda: run(L.osk_ceiling_copy(p(src), p(dst), n4, grid, st)), 5,
                      stream)
    out["hbm_copy_gbs"] = 2 * 16.0 * n4 / (t * 1e-3) / 1e9
    del dst
    sink = torch.empty(grid * 256, dtype=torch.float32, device=dev)
    t = event_time_ms(torch, lambda: run(L.osk_ceiling_read(p(src), n4, p(sink), grid, st)), 5,
                      stream)
    out["hbm_read_gbs"] = 16.0 * n4 / (t * 1e-3) / 1e9
    del src, sink
    grid = 1024
    sink = torch.empty(grid * 512, dtype=torch.float32, device=dev)
    for kind, name, k, iters in ((0, "mfma_fp32_tflops", 2, 1500), (1, "mfma_bf16_tflops", 16, 3000),
                                 (2, "mfma_fp8_tflops", 64, 1500)):
        t = event_time_ms(torch, lambda: run(L.osk_ceiling_mfma(kind, iters, grid, p(sink), st)),
                          3, stream)
        flops = grid * 8.0 * iters * 4 * (2 * 32 * 32 * k)
        out[name] = flops / (t * 1e-3) / 1e12
    for rnd, name in ((1, "lds_gather16_random"), (0, "lds_gather16_conflict_free")):
        iters = 1000
        t = event_time_ms(torch, lambda: run(L.osk_ceiling_lds_gather(iters, rnd, grid, p(sink),
                                                                      st)), 3, stream)
        reads = grid * 512.0 * iters * 8
        out[name + "_per_s"] = reads / (t * 1e-3)
    del sink
    torch.cuda.empty_cache()
    return out


def numpy_blas_sample(oracle, A_s, B_s, b, N, e, seed, keep, C_ref):
    """The sampled product C[:r, :r] in FP64 with NumPy/SciPy: the oracle's
    hash tables as a sparse n x z count-sketch matrix, the two sketches as
    sparse-dense products, the kept blocks' product through BLAS (dgemm).
    Timed from the FP32 inputs to C; the tables are built before the clock."""
    import scipy.sparse as sp
    n = A_s.shape[1]
    nblk = N + e
    h, sg = oracle.hash_tables(seed, nblk, n, b)
    kept = [i for i in range(nblk) if keep[i]]
    rows = np.tile(np.arange(n), len(kept))
    cols = np.concatenate([j * b + h[i].astype(np.int64) for j, i in enumerate(kept)])
    vals = np.concatenate([sg[i].astype(np.float64) for i in kept])
    S = sp.csc_matrix((vals, (rows, cols)), shape=(n, len(kept) * b))
    threads = os.environ.get("OMP_NUM_THREADS")
    t0 = time.perf_counter()
    A64 = A_s.astype(np.float64)
    B64 = B_s.astype(np.float64)
    At = (S.T @ A64.T).T                      # r x K b
    Bt = S.T @ B64                            # K b x r
    Cn = (np.ascontiguousarray(At) @ np.ascontiguousarray(Bt)) / len(kept)
    t = time.perf_counter() - t0
    r = A_s.shape[0]
    return {"value": 2.0 * r * n * B_s.shape[1] / t / 1e12, "unit": "TFLOP/s",
            "seconds": t, "threads": threads,
            "kind": "NumPy/SciPy FP64: sparse S (oracle's tables), BLAS dgemm over kept blocks",
            "rel_frob_vs_oracle": oracle.rel_frob(Cn, C_ref)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gram_tile_flops(sizes, K, bs, tile, mixed):
    """Flops the batched product executes (whole tiles, K*bp padded to the
    step pair) for a tile form: the work it does, against the algorithmic
    m(m+1)Kb of the upper triangles."""
    import paper_1811_02653_amd as osk
    total = 0.0
    for m, b in zip(sizes, bs):
        ld = -(-K * osk.block_stride(b) // 64) * 64
        if tile == mixed:
            T = -(-m // 256)
            big = small = 0
            for i in range(T):
                for j in range(i, T):
                    if i == j:
                        small += 3 if m - 256 * i > 128 else 1
                    elif m - 256 * j > 128:
                        big += 1
                    else:
                        small += 2
            total += 2.0 * ld * (big * 256 * 256 + small * 128 * 128)
        else:
            T = -(-m // tile)
            total += 2.0 * ld * (T * (T + 1) // 2) * tile * tile
    return total


def bench_hessian_batch(torch, osk, args, stream, reps):
    import synthetic
    from paper_1811_02653_amd.gram import MIXED, PRODUCT, PREPARE, SKETCH
    TILE_NAMES = {MIXED: "mixed", 256: "256", 128: "128"}
    count, N, e = 64, 6, 1
    sizes, As, ds = synthetic.hessian_batch_device(count, args.seed)
    keeps = [synthetic.random_keep(N, e, args.seed + k, drop=1) for k in range(count)]
    bs = [(m + 1) // 2 for m in sizes]
    gb = osk.GramBatch(As, ds, b=bs, N=N, e=e, keeps=keeps, seeds=list(range(count)),
                       stream=stream)
    tuned_ms = gb.autotune(reps=2, stream=stream)
    tile, grid = gb.config
    cands = [{"tile": TILE_NAMES[t], "grid": g, "product_ms": ms} for t, g, ms in gb.candidates]
    # the product alone for each tile form at its resident grid, re-timed
    by_tile = {}
    for t in (MIXED, 256, 128):
        gb.configure(t, 0, stream=stream)
        by_tile[TILE_NAMES[t]] = event_time_ms(torch, lambda: gb.run(PRODUCT, stream=stream),
                                               reps, stream)
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
        "tile": TILE_NAMES[tile], "grid": grid, "autotune_product_ms": tuned_ms,
        "autotune_candidates": cands,
        "product_ms_by_tile": by_tile,
        "computed_per_algorithmic_flops": {
            TILE_NAMES[t]: gram_tile_flops(sizes, K, bs, t, MIXED) / prod_flops
            for t in (MIXED, 256, 128)},
        "ms_per_batch": t_graph, "ms_per_batch_eager": t_eager,
        "hessians_per_s": count / (t_graph * 1e-3),
        "eff_tflops": exact_flops / (t_graph * 1e-3) / 1e12,
        "stages_ms": {"prepare": t_prep, "sketch": t_sketch, "product": t_prod},
        "product_roofline": {
            "kernel": "%s (FP32 v_mfma_f32_32x32x2_f32, persistent, tile %s)" %
                      ("gemm_batch_mixed" if tile == MIXED else "gemm_batch_sym", TILE_NAMES[tile]),
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
    log("hessian batch: candidates %s" % ", ".join(
        "%s/%d %.2f ms" % (c["tile"], c["grid"], c["product_ms"]) for c in cands))
    log("hessian batch: tile %s grid %d, %.3f ms per batch (graph), %.3f eager; prepare %.3f, "
        "sketch %.3f, product %.3f ms (%.1f TFLOP/s); exact %.1f ms; error mean %.3e" %
        (TILE_NAMES[tile], grid, t_graph, t_eager, t_prep, t_sketch, t_prod,
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


def profile_stage(torch, osk, args, A, B, C, ws, keep, stream):
    """One stage of the headline workload, alone, for counter collection."""
    m, n, l, b, N, e = args.m, args.n, args.l, args.b, args.N, args.e
    dev = A.device
    nst = osk.stored_count(N, e, keep, args.kept_only)
    bp = osk.block_stride(b)
    prep = osk.sketch_prepare(n, b, N, e, seed=args.seed)
    At = torch.empty((m, nst * bp), dtype=torch.float32, device=dev)
    Bt = torch.empty((l, nst * bp), dtype=torch.float32, device=dev)
    tws = torch.empty(osk.sketch_rows_workspace_bytes(n, l), dtype=torch.uint8, device=dev)
    osk.sketch_cols(A, b, N, e, seed=args.seed, keep=keep, kept_only=args.kept_only, prep=prep,
                    out=At, stream=stream)
    osk.sketch_rows(B, b, N, e, seed=args.seed, keep=keep, kept_only=args.kept_only, prep=prep,
                    out=Bt, workspace=tws, stream=stream)
    stored_keep = None if args.kept_only else keep
    QA = QB = None
    if args.profile_stage in ("gemm_bf16", "gemm_fp8"):
        prec = args.profile_stage[5:]
        QA = osk.sketch_quantize(At, b, nst, precision=prec)
        QB = osk.sketch_quantize(Bt, b, nst, precision=prec)
    # the vendor library on a product of the block product's shape (the
    # bench's precision_variants.library_reference), for its counters
    La = Lb = None
    one = torch.ones((), device=dev)
    if args.profile_stage in ("lib_bf16", "lib_fp8"):
        kb = osk.stored_count(N, e, keep, True) * bp
        La = At[:, :kb].to(torch.bfloat16)
        Lb = Bt[:, :kb].to(torch.bfloat16)
        if args.profile_stage == "lib_fp8":
            La, Lb = La.to(torch.float8_e4m3fn), Lb.to(torch.float8_e4m3fn)
    fns = {
        "step": lambda: osk.matmul(A, B, b, N, e, seed=args.seed, keep=keep,
                                   kept_only=args.kept_only, out=C, workspace=ws, stream=stream),
        "prepare": lambda: osk.sketch_prepare(n, b, N, e, seed=args.seed, stream=stream),
        "sketch_A": lambda: osk.sketch_cols(A, b, N, e, seed=args.seed, keep=keep,
                                            kept_only=args.kept_only, prep=prep, out=At,
                                            stream=stream),
        # B's columns read in place, as the whole path does for this B
        "sketch_B": lambda: osk.sketch_rows(B, b, N, e, seed=args.seed, keep=keep,
                                            kept_only=args.kept_only, prep=prep, out=Bt,
                                            workspace=None, stream=stream),
        "gemm": lambda: osk.gemm_kept(At, Bt, b, keep=stored_keep, out=C, stream=stream),
        "gemm_bf16": lambda: osk.gemm_kept_prec(QA, QB, b, nst, precision="bf16",
                                                keep=stored_keep, out=C, stream=stream),
        "gemm_fp8": lambda: osk.gemm_kept_prec(QA, QB, b, nst, precision="fp8",
                                               keep=stored_keep, out=C, stream=stream),
        "lib_bf16": lambda: torch.matmul(La, Lb.t()),
        "lib_fp8": lambda: torch._scaled_mm(La, Lb.t(), scale_a=one, scale_b=one,
                                            out_dtype=torch.float32),
    }
    fn = fns[args.profile_stage]
    torch.cuda.synchronize()
    for i in range(args.warmup + args.steps):
        fn()
        torch.cuda.synchronize()
        log("%s %d done" % (args.profile_stage, i))


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

    if args.profile_stage:
        profile_stage(torch, osk, args, A, B, C, ws, keep, stream)
        return

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
    # the whole path's prepared sketch (natural bucket order); the grouped
    # order (OS_PREPARE_GROUPED) is measured beside it
    prep = osk.sketch_prepare(n, b, N, e, seed=args.seed)
    walked, real = osk.list_entries(prep, n, b, N, e, seed=args.seed)
    grp = osk.sketch_prepare(n, b, N, e, seed=args.seed, grouped=True)
    walked_grp, _ = osk.list_entries(grp, n, b, N, e, seed=args.seed)
    At = torch.empty((m, nst * bp), dtype=torch.float32, device=dev)
    Bt = torch.empty((l, nst * bp), dtype=torch.float32, device=dev)
    stored_keep = None if args.kept_only else keep      # mask over the stored blocks
    tws = torch.empty(osk.sketch_rows_workspace_bytes(n, l), dtype=torch.uint8, device=dev)
    reps = max(3, args.steps)
    t_prep = event_time_ms(torch, lambda: osk.sketch_prepare(n, b, N, e, seed=args.seed,
                                                             stream=stream), reps, stream)
    t_prep_grp = event_time_ms(torch, lambda: osk.sketch_prepare(n, b, N, e, seed=args.seed,
                                                                 stream=stream, grouped=True),
                               reps, stream)
    t_sa_grp = event_time_ms(torch, lambda: osk.sketch_cols(A, b, N, e, seed=args.seed,
                                                            keep=keep, kept_only=args.kept_only,
                                                            prep=grp, out=At, stream=stream),
                             reps, stream)
    del grp
    t_sa = event_time_ms(torch, lambda: osk.sketch_cols(A, b, N, e, seed=args.seed, keep=keep,
                                                        kept_only=args.kept_only, prep=prep,
                                                        out=At, stream=stream),
                        reps, stream)
    # B's columns read in place (the whole path's form for a 16-byte-aligned
    # FP32 B with l and ldb multiples of 4), and transposed first, for reference
    t_sb = event_time_ms(torch, lambda: osk.sketch_rows(B, b, N, e, seed=args.seed, keep=keep,
                                                        kept_only=args.kept_only, prep=prep,
                                                        out=Bt, workspace=None, stream=stream),
                        reps, stream)
    t_sb_tr = event_time_ms(torch, lambda: osk.sketch_rows(B, b, N, e, seed=args.seed, keep=keep,
                                                           kept_only=args.kept_only, prep=prep,
                                                           out=Bt, workspace=tws, stream=stream),
                            reps, stream)
    t_gemm = event_time_ms(torch, lambda: osk.gemm_kept(At, Bt, b, keep=stored_keep, out=C,
                                                        stream=stream), reps, stream)
    gemm_flops = 2.0 * m * l * K * bp
    gemm_tflops = gemm_flops / (t_gemm * 1e-3) / 1e12
    sketch_entries_a = (m + 3) // 4 * float(n) * nst     # real list entries (4 lines each)
    sketch_bytes_a = 4.0 * (m * n + m * nst * bp)
    sketch_bytes_b = 4.0 * (n * l + l * nst * bp)
    log("stages: prepare %.3f, sketch A %.3f, sketch B %.3f (transposed first %.3f), gemm %.3f ms" %
        (t_prep, t_sa, t_sb, t_sb_tr, t_gemm))

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

    # ---- stress case: the same shapes with independent factors (A's row
    # space and B's column space unrelated), where the sketch's error is
    # about sqrt(n / (K b)) = 200 %: the product is as fast, the answer is
    # not useful (Lemma 3's scaling)
    stress = None
    if not args.no_stress:
        A3_h, B3_h = synthetic.lowrank_pair(m, n, l, args.seed, rank=64, noise=0.1,
                                            shared_factor=False)
        A3 = torch.from_numpy(A3_h).to(dev)
        B3 = torch.from_numpy(B3_h).to(dev)
        del A3_h, B3_h
        t_st = event_time_ms(torch, lambda: osk.matmul(A3, B3, b, N, e, seed=args.seed, keep=keep,
                                                       out=C, workspace=ws, stream=stream),
                             reps, stream)
        torch.cuda.synchronize()
        AB3 = torch.matmul(A3.double(), B3.double())
        Cd = C.double()
        na2, nb2 = torch.sum(A3.double() ** 2).item(), torch.sum(B3.double() ** 2).item()
        nab2 = torch.sum(AB3 ** 2).item()
        # the second moment's prediction (Lemma 1 summed over entries, K blocks)
        cross = torch.sum(torch.sum(A3.double() ** 2, dim=0) *
                          torch.sum(B3.double() ** 2, dim=1)).item()
        stress = {"workload": "as the headline, but B = P W / 8 + 0.1 G_B with P independent of A's "
                              "factor Q",
                  "ms_per_step": t_st, "eff_tflops": 2.0 * m * n * l / (t_st * 1e-3) / 1e12,
                  "rel_frob_vs_exact_fp64": (torch.sum((Cd - AB3) ** 2).item() / nab2) ** 0.5,
                  "rel_frob_predicted_rms": _predicted_rel_frob(na2, nb2, nab2, cross, K, b)}
        log("stress (independent factors): %.3f ms, error %.3f (predicted %.3f)" %
            (t_st, stress["rel_frob_vs_exact_fp64"], stress["rel_frob_predicted_rms"]))
        del A3, B3, AB3, Cd
        torch.cuda.empty_cache()
    step()

    # ---- the small validation case (A 256 x 4096, B 4096 x 256, i.i.d.
    # N(0,1), b = 256, N = 4, e = 1, one random block dropped): latency of
    # the whole path; then the same shapes with log-normal (sigma = 2) row
    # norms of A and column norms of B in every operand precision, the
    # precision workload (errors against the oracle on the same sketch are
    # taken in the CPU leg)
    small = None
    small_host = None
    if not args.no_small:
        sm, sn, sl, sb, sN, se = 256, 4096, 256, 256, 4, 1
        sseed = 3
        A1_h, B1_h = synthetic.gaussian_pair(sm, sn, sl, sseed)
        k1 = synthetic.random_keep(sN, se, sseed)
        A1, B1 = torch.from_numpy(A1_h).to(dev), torch.from_numpy(B1_h).to(dev)
        C1 = torch.empty((sm, sl), dtype=torch.float32, device=dev)
        ws1 = torch.empty(max(osk.workspace_bytes(sm, sn, sl, sb, sN, se, precision=pr)
                              for pr in osk.PRECISIONS), dtype=torch.uint8, device=dev)
        t1 = event_time_ms(torch, lambda: osk.matmul(A1, B1, sb, sN, se, seed=sseed, keep=k1,
                                                     out=C1, workspace=ws1, stream=stream),
                           100, stream)
        torch.cuda.synchronize()
        # one call captured into a HIP graph (the path enqueues kernels only)
        # and replayed back to back, for callers that replay captured steps;
        # the replay must give the eager result bit for bit
        eager = C1.clone()
        gs = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            osk.matmul(A1, B1, sb, sN, se, seed=sseed, keep=k1, out=C1, workspace=ws1, stream=gs)
        C1.fill_(float("nan"))
        t1_gpu = event_time_ms(torch, graph.replay, 100, gs)
        torch.cuda.synchronize()
        graph_ok = bool(torch.equal(C1, eager))
        del graph
        AB1 = torch.matmul(A1.double(), B1.double())
        e1 = (torch.linalg.norm(C1.double() - AB1) / torch.linalg.norm(AB1)).item()
        small_host = {"gaussian": (A1_h, B1_h, k1, C1.cpu().numpy())}
        A2_h, B2_h = synthetic.lognormal_scaled_pair(sm, sn, sl, sseed, sigma=2.0)
        A2, B2 = torch.from_numpy(A2_h).to(dev), torch.from_numpy(B2_h).to(dev)
        AB2 = torch.matmul(A2.double(), B2.double())
        logn = {}
        outs = {}
        for prec in ("fp32", "bf16", "bf16x3", "fp8", "fp8x3"):
            tq = event_time_ms(torch, lambda: osk.matmul(A2, B2, sb, sN, se, seed=sseed, keep=k1,
                                                         out=C1, workspace=ws1, stream=stream,
                                                         precision=prec), 50, stream)
            torch.cuda.synchronize()
            logn[prec] = {"us_per_step": 1e3 * tq,
                          "rel_frob_vs_exact_fp64":
                              (torch.linalg.norm(C1.double() - AB2) / torch.linalg.norm(AB2)).item()}
            outs[prec] = C1.cpu().numpy()
        small_host["lognormal"] = (A2_h, B2_h, k1, outs)
        small = {"workload": "A %dx%d . B %dx%d, i.i.d. N(0,1), b=%d, N=%d, e=%d, one random block "
                             "dropped" % (sm, sn, sn, sl, sb, sN, se),
                 "us_per_step": 1e3 * t1, "eff_tflops": 2.0 * sm * sn * sl / (t1 * 1e-3) / 1e12,
                 "us_per_step_graph_replay": 1e3 * t1_gpu, "graph_replay_bitwise_equal": graph_ok,
                 "rel_frob_vs_exact_fp64": e1,
                 "precision_lognormal": {
                     "workload": "the same shapes, A's row norms and B's column norms log-normal "
                                 "(sigma = 2)", "by_precision": logn}}
        log("small case: %.1f us per step (%.1f us as a graph replay, bitwise %s), error %.3f; "
            "log-normal: %s" %
            (1e3 * t1, 1e3 * t1_gpu, graph_ok, e1,
             {k: "%.3e" % v["rel_frob_vs_exact_fp64"] for k, v in logn.items()}))
        del A1, B1, C1, ws1, AB1, A2, B2, AB2
        torch.cuda.empty_cache()

    # ---- measured ceilings of the units the kernels are bound by
    ceil = None
    if not args.no_ceilings:
        ceil = bench_ceilings(torch, stream)
        log("ceilings: %s" % {k: round(v, 1) if v < 1e6 else "%.3e" % v for k, v in ceil.items()})

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
        # the vendor library on a product of the block product's shape
        # (m x K*bp times (l x K*bp)^T, both operands K-contiguous): BF16
        # torch.matmul (hipBLASLt) and FP8 E4M3 torch._scaled_mm with one
        # scale per tensor (the block product uses one per 64 values)
        kb = K * bp
        gl = torch.Generator(device=dev)
        gl.manual_seed(args.seed)
        La = torch.randn((m, kb), generator=gl, device=dev).to(torch.bfloat16)
        Lb = torch.randn((l, kb), generator=gl, device=dev).to(torch.bfloat16)
        lib_flops = 2.0 * m * l * kb
        t_lb = event_time_ms(torch, lambda: torch.matmul(La, Lb.t()), reps, stream)
        libref = {"shape": "%d x %d . (%d x %d)^T" % (m, kb, l, kb),
                  "bf16_matmul": {"ms": t_lb, "tflops": lib_flops / (t_lb * 1e-3) / 1e12,
                                  "frac_of_peak": lib_flops / (t_lb * 1e-3) / 1e12 /
                                  BF16_MFMA_PEAK_TFLOPS}}
        try:
            La8, Lb8 = La.to(torch.float8_e4m3fn), Lb.to(torch.float8_e4m3fn)
            one = torch.ones((), device=dev)
            t_l8 = event_time_ms(torch, lambda: torch._scaled_mm(La8, Lb8.t(), scale_a=one,
                                                                 scale_b=one,
                                                                 out_dtype=torch.float32),
                                 reps, stream)
            libref["fp8_scaled_mm_per_tensor"] = {
                "ms": t_l8, "tflops": lib_flops / (t_l8 * 1e-3) / 1e12,
                "frac_of_peak": lib_flops / (t_l8 * 1e-3) / 1e12 / FP8_MFMA_PEAK_TFLOPS}
            del La8, Lb8
        except (RuntimeError, AttributeError) as ex:
            libref["fp8_scaled_mm_per_tensor"] = {"error": str(ex)[:200]}
        precision["library_reference"] = libref
        log("library reference: %s" % libref)
        del La, Lb
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
        cpu["model"] = cpu_model()
        # a stronger CPU figure: the same sampled product with NumPy/SciPy in
        # FP64 (sparse count-sketch matrix S of the oracle's tables, then the
        # kept blocks' product through BLAS)
        cpu["blas"] = numpy_blas_sample(oracle, A_s, B_s, b, N, e, args.seed, keep, C_ref)
        log("cpu numpy/BLAS sample: %.1f s (%.3f TFLOP/s eff), agrees with the oracle to %.1e" %
            (cpu["blas"]["seconds"], cpu["blas"]["value"], cpu["blas"]["rel_frob_vs_oracle"]))
        del C_ref
        if small_host is not None:
            sb, sN, se, sseed = 256, 4, 1, 3
            A1_h, B1_h, k1, C1_h = small_host["gaussian"]
            t0 = time.perf_counter()
            ref1 = oracle.sketched_matmul(A1_h, B1_h, sb, sN, se, seed=sseed, keep=k1)
            small["oracle_ms"] = 1e3 * (time.perf_counter() - t0)
            small["rel_frob_vs_oracle"] = oracle.rel_frob(C1_h, ref1)
            A2_h, B2_h, k2, outs = small_host["lognormal"]
            ref2 = oracle.sketched_matmul(A2_h, B2_h, sb, sN, se, seed=sseed, keep=k2)
            for prec, Cq in outs.items():
                small["precision_lognormal"]["by_precision"][prec]["rel_frob_vs_oracle"] = \
                    oracle.rel_frob(Cq, ref2)
            log("small case vs oracle: %.2e; log-normal by precision vs oracle: %s" %
                (small["rel_frob_vs_oracle"],
                 {k: "%.2e" % v["rel_frob_vs_oracle"]
                  for k, v in small["precision_lognormal"]["by_precision"].items()}))

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
        "stages_ms": {"prepare": t_prep, "sketch_A": t_sa, "sketch_B": t_sb, "gemm": t_gemm,
                      "sketch_B_transposed_first": t_sb_tr},
        "sketch_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "list_entries_walked_per_real": walked / real,
            "grouped_order": {"list_entries_walked_per_real": walked_grp / real,
                              "prepare_ms": t_prep_grp, "sketch_A_ms": t_sa_grp},
            "stage_frac": (sketch_bytes_a + sketch_bytes_b) / ((t_sa + t_sb) * 1e-3) / 1e9
                          / HBM_PEAK_GBS,
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
        "small_case": small,
        "stress_independent_factors": stress,
        "ceilings": ceil,
        "vs_ceilings": None if ceil is None else {
            "gemm_fp32_frac_of_measured_mfma": gemm_tflops / ceil["mfma_fp32_tflops"],
            "sketch_A_frac_of_measured_copy": sketch_bytes_a / (t_sa * 1e-3) / 1e9
                                              / ceil["hbm_copy_gbs"],
            "sketch_B_frac_of_measured_copy": sketch_bytes_b / (t_sb * 1e-3) / 1e9
                                              / ceil["hbm_copy_gbs"],
            # the sketch's second roofline: one 16-byte LDS gather per list
            # entry (a window position of one stored block, 4 lines)
            "sketch_A_lds_entries_per_s": sketch_entries_a / (t_sa * 1e-3),
            "sketch_A_frac_of_random_lds_gather": sketch_entries_a / (t_sa * 1e-3)
                                                  / ceil["lds_gather16_random_per_s"],
            "bf16_gemm_frac_of_measured_mfma": None if precision is None else
            precision["bf16"]["gemm_tflops"] / ceil["mfma_bf16_tflops"],
            "fp8_gemm_frac_of_measured_mfma": None if precision is None else
            precision["fp8"]["gemm_tflops"] / ceil["mfma_fp8_tflops"],
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
