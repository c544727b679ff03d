"""High-level handle over the C ABI: device buffers and streams from torch.

    S = SelInv(n, colptr, rowind, perm, dtype="f64", batch=1)   # or "c128" (complex-symmetric), "h128" (Hermitian)
    S.factor(values)          # host LDL^T + upload + normalize kernels
    S.run()                   # selected inversion on the GPU (async)
    X = S.extract()           # [batch, nnz(A)] selected entries on A's pattern

dtype="lu64" takes an unsymmetric real A with a symmetric pattern: values are
[batch, 2 nnz(A)] (the stored lower entries, then their mirrors A(j, i)), the
panels and X hold two panel sets (L and X, then U^T and X^T), and extract()
returns [batch, 2 nnz(A)] in the values' order.

Everything numeric runs in the library (host C++ factorization, HIP kernels
for the rest); this module only allocates buffers and passes pointers.
"""

from __future__ import annotations

import numpy as np
import torch

from . import capi


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _bytes(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class SelInv:
    def __init__(self, n, colptr, rowind, perm=None, *, dtype="f64", batch=1, cap=256, relax=0.05,
                 sched="levels", nthreads=0, watchdog_ms=0, dense_min_c=0, dense_max_bytes=0, split_min_k=0,
                 tune_cache=None, adjoint=True, device="cuda"):
        self.n = int(n)
        if dtype not in ("f64", "float64", torch.float64, "c128", "complex128", torch.complex128, "h128", "hermitian",
                         "lu64", "lu"):
            raise ValueError(f"unknown dtype {dtype!r} (f64, c128 = complex-symmetric, h128 = Hermitian, "
                             "lu64 = unsymmetric real with a symmetric pattern)")
        self.is_hermitian = dtype in ("h128", "hermitian")
        self.is_lu = dtype in ("lu64", "lu")
        self.is_complex = self.is_hermitian or dtype in ("c128", "complex128", torch.complex128)
        self.batch = int(batch)
        self.device = device
        o = capi.selinv_default_opts()
        o.max_super = int(cap)
        o.dtype = (capi.SELINV_H128 if self.is_hermitian else capi.SELINV_LU64 if self.is_lu else
                   capi.SELINV_C128 if self.is_complex else capi.SELINV_R64)
        o.batch = self.batch
        o.sched = {"levels": capi.SCHED_LEVELS, "persistent": capi.SCHED_PERSISTENT, "push": capi.SCHED_PUSH}[sched]
        o.relax = float(relax)
        o.nthreads = int(nthreads)
        o.watchdog_ms = int(watchdog_ms)
        o.dense_min_c = int(dense_min_c)
        o.dense_max_bytes = int(dense_max_bytes)
        o.split_min_k = int(split_min_k)
        self._tune_path = None if tune_cache is None else str(tune_cache).encode()
        o.tune_cache = self._tune_path
        o.adjoint = 0 if adjoint else -1
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int64)
        self._perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
        self.h = capi.selinv_analyze(self.n, self._colptr, self._rowind, self._perm, o)
        self.view = capi.selinv_symbolic(self.h)
        self.sizes = capi.selinv_sizes(self.h)
        self.nnzA = int(self._colptr[-1])
        self.nvals = 2 * self.nnzA if self.is_lu else self.nnzA  # values (and extracted entries) per matrix
        self.panel_elems = int(self.view.panel_elems)
        self._bufs = None
        self.dtilde = None
        self.generation = 0  # successful factor() calls (the autograd binding checks it)

    # -- symbolic data (host copies) -------------------------------------------
    def symbolic(self):
        v = self.view
        ns, n = int(v.nsuper), int(v.n)
        arr = lambda p, m: np.ctypeslib.as_array(p, shape=(m,)).copy() if m > 0 else np.zeros(0, np.int64)
        rowptr = arr(v.rowptr, ns + 1)
        return {
            "n": n, "nsuper": ns, "nnzL": int(v.nnzL), "panel_elems": int(v.panel_elems),
            "perm": arr(v.perm, n), "parent": arr(v.parent, n), "colcount": arr(v.colcount, n),
            "xsuper": arr(v.xsuper, ns + 1), "sparent": arr(v.sparent, ns), "rowptr": rowptr,
            "rowind_L": arr(v.rowind_L, int(rowptr[-1])), "panel_off": arr(v.panel_off, ns),
            "seg_ptr": arr(v.seg_ptr, ns + 1), "seg_super": arr(v.seg_super, int(v.nseg)),
            "seg_start": arr(v.seg_start, int(v.nseg)), "seg_posoff": arr(v.seg_posoff, int(v.nseg)),
            "posarr": arr(v.posarr, int(v.nposarr)),
            "flops": float(v.flops), "flops_exact": float(v.flops_exact), "depth": int(v.depth),
            "tuned_nodes": int(v.tuned_nodes),
        }

    # -- buffers -----------------------------------------------------------------
    @property
    def scalar_dtype(self):
        return torch.complex128 if self.is_complex else torch.float64

    def _alloc(self, want_dtilde):
        if self._bufs is None:
            s = self.sizes
            self._bufs = {
                "panels": _bytes(s.panels_bytes, self.device),
                "x": _bytes(s.x_bytes, self.device),
                "work": _bytes(s.work_bytes, self.device),
            }
        if want_dtilde and self.dtilde is None:
            self.dtilde = _bytes(self.sizes.dtilde_bytes, self.device)

    def panels_view(self, which="x"):
        """[batch, panel_elems] view of the panels or of X."""
        b = self._bufs[which]
        nb = self.batch * self.panel_elems * (16 if self.is_complex else 8)
        return b[:nb].view(self.scalar_dtype).view(self.batch, self.panel_elems)

    def packed_index(self):
        """Element indices of the unpadded concatenation of the panels (LU:
        of the first panel set, then of the second)."""
        if getattr(self, "_packed", None) is None:
            sym = self.symbolic()
            ws = np.diff(sym["xsuper"])
            cs = np.diff(sym["rowptr"])
            sizes = (ws + cs) * ws
            starts = sym["panel_off"]
            idx = np.concatenate([np.arange(st, st + sz) for st, sz in zip(starts, sizes)]) if len(sizes) else np.zeros(0, np.int64)
            if self.is_lu:
                idx = np.concatenate([idx, idx + self.panel_elems // 2])
            self._packed = idx
        return self._packed

    def to_host(self, which="x"):
        """[batch, sum_K (s+c) s] numpy copy of X (or the panels), panels packed back to back."""
        full = self.panels_view(which).cpu().numpy()
        return full[:, self.packed_index()]

    # -- numeric -----------------------------------------------------------------
    def _values_host(self, values):
        if isinstance(values, torch.Tensor):
            values = values.detach().cpu().numpy()
        dt = np.complex128 if self.is_complex else np.float64
        v = np.ascontiguousarray(np.asarray(values).reshape(self.batch, self.nvals), dtype=dt)
        return v

    def _values_device(self, values):
        v = torch.as_tensor(values)
        return v.to(device=self.device, dtype=self.scalar_dtype).reshape(self.batch, self.nvals).contiguous()

    def factor(self, values, want_dtilde=False, on_device=False):
        """LDL^T of every matrix (host C++, or on the GPU with on_device=True),
        then the normalization kernels into the panels."""
        self._alloc(want_dtilde)
        dt = self.dtilde if want_dtilde else None
        if on_device:
            v = self._values_device(values)
            self._vals_keep = v
            P, W = self._bufs["panels"], self._bufs["work"]
            capi.selinv_factor_device(self.h, v, P, W, _stream())
            capi.selinv_normalize(self.h, P, P, W, dt, _stream())
        else:
            v = self._values_host(values)
            self._vals_keep = v
            capi.selinv_factor(self.h, v, self._bufs["panels"], self._bufs["work"], dt, _stream())
        self.generation += 1

    def factor_device(self, values, out=None):
        """LDL^T panels of every matrix computed on the GPU ([batch, panel_elems]
        device tensor; strict lower L_KK, D_K on the diagonal, L_{C,K} below)."""
        self._alloc(False)
        v = self._values_device(values)
        if out is None:
            out = torch.empty((self.batch, self.panel_elems), dtype=self.scalar_dtype, device=self.device)
        capi.selinv_factor_device(self.h, v, out, self._bufs["work"], _stream())
        return out

    def factor_host(self, values):
        """Host LDL^T panels only (numpy [batch, panel_elems])."""
        v = self._values_host(values)
        out = np.zeros((self.batch, self.panel_elems), dtype=np.complex128 if self.is_complex else np.float64)
        capi.selinv_factor_host(self.h, v, out)
        return out

    def run(self):
        capi.selinv_run(self.h, self._bufs["panels"], self._bufs["x"], self._bufs["work"], _stream())

    def trace_run(self):
        """Run once with per-item tracing; returns int64 [n_tickets, 8] rows
        {item, workgroup, t_ticket, t_start, t_end, 0, 0, 0} in wall-clock
        ticks: ticket drawn, dependencies met and item started, item done."""
        tr = torch.zeros(self.sizes.trace_bytes // 8, dtype=torch.int64, device=self.device)
        capi.selinv_trace(self.h, tr)
        self.run()
        self.sync()
        capi.selinv_trace(self.h, None)
        return tr.view(-1, 8).cpu().numpy()

    def sync(self):
        capi.selinv_sync(self.h, _stream())

    def extract(self, out=None):
        if out is None:
            out = torch.empty((self.batch, self.nvals), dtype=self.scalar_dtype, device=self.device)
        capi.selinv_extract(self.h, self._bufs["x"], self._bufs["work"], out, _stream())
        return out

    def scatter(self, vals):
        """[batch, panel_elems] device tensor: zeros, with vals ([batch, nnz(A)],
        on A's pattern) at the positions of A's entries (the transpose of extract)."""
        out = torch.empty((self.batch, self.panel_elems), dtype=self.scalar_dtype, device=self.device)
        capi.selinv_scatter(self.h, vals, self._bufs["work"], out, _stream())
        return out

    def backward(self, xbar, wlogdet=None, abar=None):
        """Adjoint: xbar [batch, panel_elems] device tensor, dloss/dx for the
        stored selected entries (overwritten); wlogdet: None or a [batch] device
        tensor of the scalar dtype, dloss/d(log det A_l); returns dloss/da on A's
        pattern [batch, nnz(A)].  For complex-symmetric A these are holomorphic
        derivatives (plain transposes, no conjugation).  Needs
        factor(..., want_dtilde=True) and run() first (the library returns
        ESTATE otherwise) and a context built with adjoint=True."""
        if abar is None:
            abar = torch.empty((self.batch, self.nnzA), dtype=self.scalar_dtype, device=self.device)
        capi.selinv_backward(self.h, self._bufs["panels"], self._bufs["x"], self.dtilde, xbar, wlogdet,
                             self._bufs["work"], abar, _stream())
        return abar

    def logdet(self):
        if self._bufs is not None:
            self.sync()  # a device factorization reports its log det at the next sync
        out = np.zeros(self.batch * (2 if self.is_complex else 1))
        capi.selinv_logdet(self.h, out)
        if self.is_complex:
            return out[0::2] + 1j * out[1::2]
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            capi.selinv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
