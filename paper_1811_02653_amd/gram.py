"""Batched sketched Gram matrices (the ``os_gram_*`` entry points).

For problems k = 0 .. count-1 with A_k (m_k x n_k, row-major FP32 on the
device) and nonnegative diagonal weights d_k (length n_k, or None for ones):

    H_k = (1/K_k) * sum over kept blocks i of (A_k D_k^{1/2} S_i)(A_k D_k^{1/2} S_i)^T

the sketched Hessian of the log-barrier interior-point method (Section 5.2,
Eq. (int_point) and the Hessian after it, with A_k the constraint matrix
transposed and d_k = 1/(b - a_i x)^2).  One plan holds the whole batch; a run
prepares and sketches every problem, then computes every H_k in one
persistent launch.  Argument marshalling only: all steps run in the library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import (OversketchError, _GramCandidate, _GramProblem, _check, _mask, _ptr, _require_cuda,
               _row_major, _sketch, _stream, _torch, lib)


# stages of a run (OS_GRAM_* in oversketch.h)
PREPARE, SKETCH, PRODUCT = 1, 2, 4
ALL = PREPARE | SKETCH | PRODUCT
# tile form: 256 tiles inside each triangle, pairs of 128 tiles along its
# diagonal and ragged edge (OS_GRAM_MIXED)
MIXED = 1


class GramGraph:
    """An executable HIP graph of one batch run (os_gram_graph_create)."""

    def __init__(self, handle, owner):
        self._h = handle
        self._owner = owner       # keeps the plan, its tensors and workspace alive

    def launch(self, stream=None):
        if not self._h:
            raise OversketchError("graph already released")
        _check(lib().os_graph_launch(self._h, _stream(stream)), "os_graph_launch")

    def close(self):
        if self._h:
            lib().os_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GramBatch:
    """A planned batch of sketched Gram matrices.

    A_list: CUDA float32 tensors (m_k x n_k, unit column stride); d_list: CUDA
    float32 vectors (n_k) or None; b: block width per problem (int or list);
    N, e: blocks kept / extra (ints or lists); seeds: hash seed per problem
    (default k); keeps: per problem a host mask over N+e blocks or None
    (= blocks [0, N)); full: write H whole (else only the tiles on or above
    the diagonal); out: optional list of CUDA float32 m_k x m_k tensors.
    The plan is configured with tile form `tile` (256, 128 or MIXED: 256
    tiles inside each triangle, pairs of 128 tiles along its diagonal and
    ragged edge) and `grid` persistent workgroups (0 = the device's resident
    count); ``autotune()`` picks the form and grid by timing.
    """

    def __init__(self, A_list, d_list=None, b=None, N=6, e=1, seeds=None, keeps=None, full=True,
                 out=None, tile=MIXED, grid=0, hs=None, sigmas=None, stream=None):
        torch = _torch()
        count = len(A_list)
        if count < 1:
            raise OversketchError("empty batch")

        def per(x, name):
            if isinstance(x, (list, tuple)):
                if len(x) != count:
                    raise OversketchError("%s needs %d entries" % (name, count))
                return list(x)
            return [x] * count

        d_list = per(d_list, "d_list")
        bs = per(b, "b")
        Ns, es = per(N, "N"), per(e, "e")
        seeds = list(range(count)) if seeds is None else per(seeds, "seeds")
        keeps = per(keeps, "keeps")
        hs, sigmas = per(hs, "hs"), per(sigmas, "sigmas")
        self.A, self.d, self.H, self._keep = [], [], [], []
        self._tables = []
        probs = (_GramProblem * count)()
        for k in range(count):
            A = A_list[k]
            _require_cuda(A, "A[%d]" % k, torch.float32)
            m, n, lda = _row_major(A, "A[%d]" % k)
            if bs[k] is None:
                raise OversketchError("b is required")
            p = probs[k]
            p.sk = _sketch(bs[k], Ns[k], es[k], seeds[k], hs[k], sigmas[k], n)
            p.A, p.lda, p.m, p.n = A.data_ptr(), lda, m, n
            dk = d_list[k]
            if dk is not None:
                _require_cuda(dk, "d[%d]" % k, torch.float32)
                if dk.dim() != 1 or dk.shape[0] != n or dk.stride(0) != 1:
                    raise OversketchError("d[%d] must be a contiguous vector of length n" % k)
                p.d = dk.data_ptr()
            else:
                p.d = None
            arr, kp = _mask(keeps[k], int(Ns[k]) + int(es[k]))
            p.keep = kp
            if out is not None:
                Hk = out[k]
                _require_cuda(Hk, "out[%d]" % k, torch.float32)
                if tuple(Hk.shape) != (m, m):
                    raise OversketchError("out[%d] must be %d x %d" % (k, m, m))
            else:
                Hk = torch.empty((m, m), dtype=torch.float32, device=A.device)
            _, _, ldh = _row_major(Hk, "out[%d]" % k)
            p.H, p.ldh = Hk.data_ptr(), ldh
            self.A.append(A)
            self.d.append(dk)
            self.H.append(Hk)
            self._keep.append(arr)
            self._tables.append((hs[k], sigmas[k]))
        L = lib()
        h = ctypes.c_void_p()
        _check(L.os_gram_plan_create(probs, count, 1 if full else 0, ctypes.byref(h)),
               "os_gram_plan_create")
        self._plan = h
        nbytes = int(L.os_gram_workspace_bytes(h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A_list[0].device)
        self.full = bool(full)
        self.configure(tile, grid, stream)

    # -- plan state -------------------------------------------------------
    def _args(self):
        return self._plan, _ptr(self.workspace), self.workspace.numel()

    @property
    def workspace_bytes(self) -> int:
        return self.workspace.numel()

    @property
    def config(self):
        """(tile form, grid) of the current configuration."""
        t, g = ctypes.c_int32(), ctypes.c_int32()
        lib().os_gram_config(self._plan, ctypes.byref(t), ctypes.byref(g))
        return t.value, g.value

    def configure(self, tile=MIXED, grid=0, stream=None):
        plan, ws, nb = self._args()
        _check(lib().os_gram_configure(plan, int(tile), int(grid), ws, nb, _stream(stream)),
               "os_gram_configure")

    def autotune(self, reps=2, stream=None) -> float:
        """Times the product for each tile form and grid (after one run of
        the earlier stages) and keeps the fastest; returns its average
        milliseconds per product run.  The timings are left in
        ``self.candidates`` as (tile, grid, ms) tuples."""
        plan, ws, nb = self._args()
        ms = ctypes.c_float()
        cap = 16
        cands = (_GramCandidate * cap)()
        count = ctypes.c_int32()
        _check(lib().os_gram_autotune_ex(plan, int(reps), ws, nb, _stream(stream), cands, cap,
                                         ctypes.byref(count), ctypes.byref(ms)),
               "os_gram_autotune_ex")
        self.candidates = [(c.tile, c.grid, float(c.ms)) for c in cands[:min(count.value, cap)]]
        return float(ms.value)

    # -- execution --------------------------------------------------------
    def run(self, stages=ALL, stream=None):
        """Enqueues the given stages (PREPARE | SKETCH | PRODUCT, default
        all); returns the list of H tensors."""
        plan, ws, nb = self._args()
        _check(lib().os_gram_run(plan, int(stages), ws, nb, _stream(stream)), "os_gram_run")
        return self.H

    def graph(self, stages=ALL, stream=None) -> GramGraph:
        """Captures one run of the given stages into an executable graph.
        `stream` must be a created (non-default) stream; by default a
        private one is used."""
        torch = _torch()
        s = stream if stream is not None else torch.cuda.Stream(device=self.workspace.device)
        plan, ws, nb = self._args()
        g = ctypes.c_void_p()
        cur = torch.cuda.current_stream(self.workspace.device)
        s.wait_stream(cur)
        _check(lib().os_gram_graph_create(plan, int(stages), ws, nb,
                                          ctypes.c_void_p(s.cuda_stream), ctypes.byref(g)),
               "os_gram_graph_create")
        return GramGraph(g.value, self)

    def close(self):
        if getattr(self, "_plan", None):
            lib().os_gram_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
