"""MI355X blocked sparse LU with structure-aware irregular blocking.

Thin Python binding of the C ABI (``include/slu.h``).  Host arrays are numpy;
device buffers are torch tensors used only for memory and streams.  All the
numerical work runs in the HIP kernels of ``libslu.so``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import (SLU_BLOCK_IRREGULAR, SLU_BLOCK_REGULAR, SLU_ORDER_GRID_ND,
                   SLU_ORDER_NATURAL, SLU_ORDER_USER, SluError, ZeroPivot, check, lib)

__all__ = ["SparseLU", "SluError", "ZeroPivot", "lib", "solve"]


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(name, t, device, numel=None, rows=None):
    """Raise ValueError unless t is a float64 tensor on the bound device
    (contiguous when numel is given: it is passed as a flat array; with rows,
    a vector of that length or a matrix of that many rows)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64:
        raise ValueError("%s must be float64, got %s" % (name, t.dtype))
    if not t.is_cuda or (device is not None and t.device != device):
        raise ValueError("%s must live on %s, got %s" % (name, device, t.device))
    if numel is not None:
        if t.numel() != numel or not t.is_contiguous():
            raise ValueError("%s must be a contiguous tensor of %d entries, got shape %s"
                             % (name, numel, tuple(t.shape)))
    if rows is not None:
        if t.dim() not in (1, 2) or t.shape[0] != rows:
            raise ValueError("%s must have %d rows (a vector or an n x nrhs matrix), got shape %s"
                             % (name, rows, tuple(t.shape)))


class SparseLU:
    """One analyzed pattern: ``slu_analyze`` at construction, then
    ``bind`` (workspace), ``factor``, ``solve`` / ``solve_transpose``."""

    def __init__(self, n, rowptr, colidx, ordering="natural", grid_dims=None, perm=None,
                 blocking="irregular", block_size=0, sample_points=1000, step=2, max_num=3,
                 advance=1, schedule="waves"):
        self.n = int(n)
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        opt = _abi.slu_options()
        lib.slu_default_options(ctypes.byref(opt))
        opt.sample_points, opt.step, opt.max_num, opt.advance = sample_points, step, max_num, advance
        opt.blocking = {"irregular": SLU_BLOCK_IRREGULAR, "regular": SLU_BLOCK_REGULAR}[blocking]
        opt.regular_block = int(block_size)
        opt.schedule = {"waves": _abi.SLU_SCHEDULE_WAVES, "levels": _abi.SLU_SCHEDULE_LEVELS}[schedule]
        self._perm_in = None
        if ordering == "natural":
            opt.ordering = SLU_ORDER_NATURAL
        elif ordering == "grid_nd":
            opt.ordering = SLU_ORDER_GRID_ND
            dims = tuple(int(v) for v in grid_dims) + (1,) * (3 - len(grid_dims))
            for d in range(3):
                opt.grid_dims[d] = dims[d]
        elif ordering == "graph_nd":
            opt.ordering = _abi.SLU_ORDER_GRAPH_ND
        elif ordering == "user":
            opt.ordering = SLU_ORDER_USER
            self._perm_in = np.ascontiguousarray(perm, dtype=np.int32)
            opt.user_perm = self._perm_in.ctypes.data
        else:
            raise ValueError("unknown ordering %r" % ordering)
        h = ctypes.c_void_p()
        check(lib.slu_analyze(self.n, _vp(self._rowptr), _vp(self._colidx), ctypes.byref(opt),
                              ctypes.byref(h)), "slu_analyze")
        self._h = h
        self._ws = None
        self.device = None
        self._serial = 0          # bumped by every successful factor

    @classmethod
    def batch(cls, systems, ordering="natural", grid_dims=None, blocking="irregular", block_size=0,
              sample_points=1000, step=2, max_num=3, advance=1, schedule="waves"):
        """One handle over independent systems [(n, rowptr, colidx), ...]
        factored together (``slu_analyze_batch``); values, right-hand sides
        and solutions are the systems' arrays concatenated in order.
        ``grid_dims``: one (nx, ny, nz) per system for ``"grid_nd"``."""
        self = cls.__new__(cls)
        ns = len(systems)
        nvec = np.array([int(s[0]) for s in systems], dtype=np.int64)
        rps = [np.ascontiguousarray(s[1], dtype=np.int64) for s in systems]
        cis = [np.ascontiguousarray(s[2], dtype=np.int32) for s in systems]
        opt = _abi.slu_options()
        lib.slu_default_options(ctypes.byref(opt))
        opt.sample_points, opt.step, opt.max_num, opt.advance = sample_points, step, max_num, advance
        opt.blocking = {"irregular": SLU_BLOCK_IRREGULAR, "regular": SLU_BLOCK_REGULAR}[blocking]
        opt.regular_block = int(block_size)
        opt.schedule = {"waves": _abi.SLU_SCHEDULE_WAVES, "levels": _abi.SLU_SCHEDULE_LEVELS}[schedule]
        opt.ordering = {"natural": SLU_ORDER_NATURAL, "grid_nd": SLU_ORDER_GRID_ND,
                        "graph_nd": _abi.SLU_ORDER_GRAPH_ND}[ordering]
        dims = None
        if ordering == "grid_nd":
            dims = np.ascontiguousarray([tuple(int(x) for x in g) + (1,) * (3 - len(g)) for g in grid_dims],
                                        dtype=np.int32).reshape(-1)
        rp_ptrs = (ctypes.c_void_p * ns)(*[a.ctypes.data for a in rps])
        ci_ptrs = (ctypes.c_void_p * ns)(*[a.ctypes.data if a.size else 0 for a in cis])
        h = ctypes.c_void_p()
        check(lib.slu_analyze_batch(ns, _vp(nvec), ctypes.cast(rp_ptrs, ctypes.c_void_p),
                                    ctypes.cast(ci_ptrs, ctypes.c_void_p), _vp(dims), ctypes.byref(opt),
                                    ctypes.byref(h)), "slu_analyze_batch")
        self.n = int(nvec.sum())
        offs = np.concatenate([[0], np.cumsum([int(r[-1]) for r in rps])])
        self._rowptr = np.concatenate([[0]] + [r[1:] + o for r, o in zip(rps, offs[:-1])]).astype(np.int64)
        self._colidx = None
        self._perm_in = None
        self._h = h
        self._ws = None
        self.device = None
        self._serial = 0
        self.sizes = nvec
        return self

    # ---------------------------------------------------------------- info
    def info(self):
        inf = _abi.slu_info()
        check(lib.slu_get_info(self._h, ctypes.byref(inf)), "slu_get_info")
        return {name: getattr(inf, name) for name, _ in _abi.slu_info._fields_}

    def perm(self):
        out = np.empty(self.n, dtype=np.int32)
        check(lib.slu_get_perm(self._h, _vp(out)), "slu_get_perm")
        return out

    def blockptr(self):
        out = np.empty(self.n + 1, dtype=np.int64)
        check(lib.slu_get_blockptr(self._h, _vp(out)), "slu_get_blockptr")
        return out

    def blocking(self):
        out = np.empty(self.info()["nblocks"] + 1, dtype=np.int64)
        check(lib.slu_get_blocking(self._h, _vp(out)), "slu_get_blocking")
        return out

    def pattern(self):
        colptr = np.empty(self.n + 1, dtype=np.int64)
        nnz_s = self.info()["nnz_s"]
        rowidx = np.empty((nnz_s + self.n) // 2, dtype=np.int32)
        check(lib.slu_get_pattern(self._h, _vp(colptr), _vp(rowidx)), "slu_get_pattern")
        return colptr, rowidx

    def workspace_size(self):
        sz = ctypes.c_size_t()
        check(lib.slu_workspace_size(self._h, ctypes.byref(sz)), "slu_workspace_size")
        return int(sz.value)

    # -------------------------------------------------------------- device
    def bind(self, device="cuda", stream=None, workspace=None):
        import torch
        nbytes = self.workspace_size()
        if workspace is None:
            workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 device tensor")
        check(lib.slu_bind_workspace(self._h, _dptr(workspace), workspace.numel(), _stream(stream)),
              "slu_bind_workspace")
        self._ws = workspace
        self.device = workspace.device
        return self

    def _nnz(self):
        return int(self.info()["nnz_a"])

    def _bound(self):
        if self._ws is None:
            raise RuntimeError("bind() a workspace first")
        return self.device

    def factor(self, values, stream=None):
        _check_dev("values", values, self._bound(), numel=self._nnz())
        self._serial += 1
        rc = lib.slu_factor(self._h, _dptr(values), _stream(stream))
        if rc == _abi.SLU_ZERO_PIVOT:
            raise ZeroPivot(self.info()["zero_pivot_col"])
        check(rc, "slu_factor")

    def _solve(self, fn, B, X, stream):
        import torch
        dev = self._bound()
        _check_dev("B", B, dev, rows=self.n)
        if X is not None:
            _check_dev("X", X, dev, rows=self.n)
            if X.shape != B.shape:
                raise ValueError("X must have the shape of B %s, got %s" % (tuple(B.shape), tuple(X.shape)))
        vec = B.dim() == 1
        Bm = B.reshape(-1, 1) if vec else B
        nrhs = Bm.shape[1]
        # column-major n x nrhs: a (nrhs, n) row-major tensor viewed transposed
        Bc = Bm.t().contiguous()
        if X is None:
            Xc = torch.empty_like(Bc)
        else:
            Xc = X.reshape(-1, 1).t().contiguous() if vec else X.t().contiguous()
        check(fn(self._h, _dptr(Bc), _dptr(Xc), nrhs, self.n, _stream(stream)), fn.__name__)
        out = Xc.t()
        return out.reshape(-1) if vec else out

    def solve(self, B, X=None, stream=None):
        return self._solve(lib.slu_solve, B, X, stream)

    def solve_transpose(self, B, X=None, stream=None):
        return self._solve(lib.slu_solve_transpose, B, X, stream)

    def solve_noalloc(self, B, X=None, transpose=False, stream=None):
        """``slu_solve_noalloc``: the solve (or transpose solve) with its
        work block in the library's fixed device scratch."""
        t = 1 if transpose else 0

        def fn(h, Bp, Xp, nrhs, ld, st):
            return lib.slu_solve_noalloc(h, Bp, Xp, nrhs, ld, t, st)
        fn.__name__ = "slu_solve_noalloc"
        return self._solve(fn, B, X, stream)

    def set_graph(self, enable=True):
        """Capture the factorization's launches into a HIP graph and replay
        it in later factors (see ``slu_set_graph``)."""
        check(lib.slu_set_graph(self._h, 1 if enable else 0), "slu_set_graph")

    def set_getrf_split(self, min_work):
        """Trailing work from which a wave's GETRF is split into a panel and
        a chip-wide trailing-update launch per column chunk (see
        ``slu_set_getrf_split``; 0 splits every wave with a chunked block)."""
        check(lib.slu_set_getrf_split(self._h, float(min_work)), "slu_set_getrf_split")

    def set_getrf_tiled(self, min_rows):
        """Waves whose largest diagonal block has at least ``min_rows`` rows
        take the tiled GETRF (see ``slu_set_getrf_tiled``; 0: none)."""
        check(lib.slu_set_getrf_tiled(self._h, int(min_rows)), "slu_set_getrf_tiled")

    def set_panel_blocked(self, enable=True):
        """Blocked panel solves for wide coupled triangles (see
        ``slu_set_panel_blocked``)."""
        check(lib.slu_set_panel_blocked(self._h, 1 if enable else 0), "slu_set_panel_blocked")

    def set_lookahead(self, enable=True, max_groups=512):
        """Schur updates that reach only later waves on a second stream,
        overlapping the next wave's diagonal and panel work, in launches of
        at most ``max_groups`` workgroups (see ``slu_set_lookahead``)."""
        check(lib.slu_set_lookahead(self._h, 1 if enable else 0, int(max_groups)), "slu_set_lookahead")

    def autotune(self, values, reps=2, stream=None):
        """Try the library's launch-shape settings on these values and keep
        the fastest (``slu_autotune``); returns the table of settings tried
        with their median factor times, the chosen one first."""
        _check_dev("values", values, self._bound(), numel=self._nnz())
        cap = 16
        table = (_abi.slu_tune_entry * cap)()
        cnt = ctypes.c_int(0)
        rc = lib.slu_autotune(self._h, _dptr(values), int(reps), ctypes.cast(table, ctypes.c_void_p), cap,
                              ctypes.byref(cnt), _stream(stream))
        if rc == _abi.SLU_ZERO_PIVOT:
            raise ZeroPivot(self.info()["zero_pivot_col"])
        check(rc, "slu_autotune")
        self._serial += 1
        rows = [{name: getattr(table[i], name) for name, _ in _abi.slu_tune_entry._fields_}
                for i in range(min(cnt.value, cap))]
        rows.sort(key=lambda r: r["ms"])
        return rows

    def set_solve_tiled(self, min_rows, min_sparse_rows=64):
        """Tiled diagonal solves for waves with blocks of at least ``min_rows``
        rows (see ``slu_set_solve_tiled``; 0: never)."""
        check(lib.slu_set_solve_tiled(self._h, int(min_rows), int(min_sparse_rows)), "slu_set_solve_tiled")

    def set_getrf_tile(self, tile):
        """Tile edge of the tiled GETRF, 16 or 32 (see ``slu_set_getrf_tile``)."""
        check(lib.slu_set_getrf_tile(self._h, int(tile)), "slu_set_getrf_tile")

    def set_precision(self, precision):
        """``"fp64"`` (default) or ``"fp32"`` (Schur updates in FP32 on the
        matrix cores, see ``slu_set_precision``) for later factorizations."""
        code = {"fp64": _abi.SLU_PRECISION_FP64, "fp32": _abi.SLU_PRECISION_FP32}[precision]
        check(lib.slu_set_precision(self._h, code), "slu_set_precision")

    def solve_refined(self, values, B, tol=1e-12, maxit=10, stream=None):
        """FP64 iterative refinement on the current factors; returns
        (X, corrections applied, per-column backward errors, converged)."""
        import torch
        dev = self._bound()
        _check_dev("values", values, dev, numel=self._nnz())
        _check_dev("B", B, dev, rows=self.n)
        vec = B.dim() == 1
        Bc = (B.reshape(-1, 1) if vec else B).t().contiguous()
        Xc = torch.empty_like(Bc)
        nrhs = Bc.shape[0]
        eta = np.empty(nrhs, dtype=np.float64)
        it = ctypes.c_int(0)
        rc = lib.slu_solve_refined(self._h, _dptr(values), _dptr(Bc), _dptr(Xc), nrhs, self.n, float(tol),
                                   int(maxit), ctypes.byref(it), _vp(eta), _stream(stream))
        if rc != _abi.SLU_NOT_CONVERGED:
            check(rc, "slu_solve_refined")
        out = Xc.t()
        return (out.reshape(-1) if vec else out), it.value, eta, rc == _abi.SLU_OK

    def value_gradient(self, G, X, stream=None):
        """-G X^T restricted to A's pattern, in the CSR order of the
        analysis (see ``slu_value_gradient``)."""
        import torch
        dev = self._bound()
        _check_dev("G", G, dev, rows=self.n)
        _check_dev("X", X, dev, rows=self.n)
        if G.shape != X.shape:
            raise ValueError("G and X must have one shape, got %s and %s" % (tuple(G.shape), tuple(X.shape)))
        Gc = (G.reshape(-1, 1) if G.dim() == 1 else G).t().contiguous()
        Xc = (X.reshape(-1, 1) if X.dim() == 1 else X).t().contiguous()
        nnz = int(self._rowptr[-1])
        out = torch.empty(nnz, dtype=torch.float64, device=Gc.device)
        check(lib.slu_value_gradient(self._h, _dptr(Gc), _dptr(Xc), Gc.shape[0], self.n, _dptr(out),
                                     _stream(stream)), "slu_value_gradient")
        return out

    def backward_error(self, values, B, X, transpose=False, stream=None):
        dev = self._bound()
        _check_dev("values", values, dev, numel=self._nnz())
        _check_dev("B", B, dev, rows=self.n)
        _check_dev("X", X, dev, rows=self.n)
        if B.shape != X.shape:
            raise ValueError("B and X must have one shape, got %s and %s" % (tuple(B.shape), tuple(X.shape)))
        vec = B.dim() == 1
        Bc = (B.reshape(-1, 1) if vec else B).t().contiguous()
        Xc = (X.reshape(-1, 1) if vec else X).t().contiguous()
        nrhs = Bc.shape[0]
        eta = np.empty(nrhs, dtype=np.float64)
        check(lib.slu_backward_error(self._h, _dptr(values), _dptr(Bc), _dptr(Xc), nrhs, self.n,
                                     1 if transpose else 0, _vp(eta), _stream(stream)),
              "slu_backward_error")
        return eta

    def factors(self, stream=None):
        """(lval, uval) on the lower CSC of S (see ``slu_get_factors``)."""
        colptr, _ = self.pattern()
        lv = np.empty(int(colptr[-1]), dtype=np.float64)
        uv = np.empty(int(colptr[-1]), dtype=np.float64)
        check(lib.slu_get_factors(self._h, _vp(lv), _vp(uv), _stream(stream)), "slu_get_factors")
        return lv, uv

    def set_profiling(self, enable=True):
        check(lib.slu_set_profiling(self._h, 1 if enable else 0), "slu_set_profiling")

    def kernel_times(self):
        """{kernel: (ms, launches)} of the last factor with profiling on."""
        ms = np.zeros(len(_abi.KERNELS), dtype=np.float64)
        nl = np.zeros(len(_abi.KERNELS), dtype=np.int64)
        check(lib.slu_get_kernel_times(self._h, _vp(ms), _vp(nl)), "slu_get_kernel_times")
        return {k: (float(ms[i]), int(nl[i])) for i, k in enumerate(_abi.KERNELS)}

    def close(self):
        if getattr(self, "_h", None):
            lib.slu_free(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



def solve(lu, values, B):
    """Differentiable x = A^{-1} B for the pattern analyzed by ``lu`` (bound
    to a workspace): factors A with ``values`` (device float64, CSR order of
    the analysis) and solves; gradients flow to ``values`` and ``B`` (see
    ``paper_2512_04389_amd.autograd``)."""
    from .autograd import SparseSolve
    return SparseSolve.apply(values, B, lu)
