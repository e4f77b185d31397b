"""Python binding of the local FusedMM library: sparse pattern objects and the
autograd-enabled operations.

PyTorch supplies device memory and the current stream; every arithmetic step runs
in libfmm.so (see include/fmm.h).  Operations (Section II of the paper):

  sddmm(P, A, B)      R = S * (A B^T) at S's stored entries, CSR order (Eq. (1))
  spmm_a(P, B, w)     S B   (or W B with stored values w)
  spmm_b(P, A, w)     S^T A (or W^T A)
  fusedmm_a(P, A, B)  SpMMA(SDDMM(A, B, S), B)
  fusedmm_b(P, A, B)  SpMMB(SDDMM(A, B, S), A), on the stored transposed copy

A and B may be float32, bfloat16 (storage; float32 accumulation and outputs) or
float64.  Gradients flow to A, B (and to w for the SpMMs); S's values are constants.
"""
from __future__ import annotations

import copy
import ctypes
from typing import Optional

import numpy as np
import torch

from . import _capi as C

__all__ = ["Pattern", "sddmm", "spmm_a", "spmm_b", "fusedmm_a", "fusedmm_b", "to_bf16", "set_tuning",
           "device_info", "dtype_code", "BatchPlan", "gat_scores", "gat_forward", "gat_edge_values",
           "gat_forward_unfused", "gat_backward", "gat", "gat_autotune", "cg_lines", "als_residual",
           "als_sweep", "stream_copy", "stream_read", "stream_gather"]

DEFAULT_LONG_LEN = 128
DEFAULT_CHUNK = 128
SPLIT_CANDIDATES = (256, 128, 64)
# Gather hints keep the rows of the longest minor lines in cache: as many rows as this
# many bytes of gathered rows hold (the L2 of the 8 XCDs together: 32 MiB).
HINT_BYTES = 32 << 20
_NO_SPLIT = (1 << 31) - 1


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def dtype_code(t: torch.Tensor) -> int:
    """The library dtype code of a dense operand (FMM_F32, FMM_BF16 or FMM_F64)."""
    if t.dtype == torch.float32:
        return C.FMM_F32
    if t.dtype == torch.bfloat16:
        return C.FMM_BF16
    if t.dtype == torch.float64:
        return C.FMM_F64
    raise TypeError(f"unsupported dense dtype {t.dtype}")


def _out_dtype(code: int):
    return torch.float64 if code == C.FMM_F64 else torch.float32


def _dev_tensor(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


def _check_dense(name, t, rows, r, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, pattern on {device}")
    if t.dim() != 2 or t.shape[0] != rows or (r is not None and t.shape[1] != r):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected ({rows}, {r if r is not None else 'r'})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")


def _check_buf(name, t, device, dtype, shape=None, min_numel=None):
    """A caller-supplied output or workspace tensor: on the pattern's device, of the dtype
    the kernel writes or reads, contiguous, and of the right shape (or at least min_numel
    elements), so that no launch touches memory outside it."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, pattern on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {min_numel}")
    return t


class Pattern:
    """A sparse matrix S (m x n) resident on the GPU in both orientations.

    Holds the canonical CSR (rowptr, colidx, val), the stored transposed copy
    (colptr, rowidx, valT, perm) built by the library's GPU transpose, and, where
    some line has more than ``long_len`` entries, the split schedules of both
    orientations, and each orientation's line processing order by decreasing length
    (fmm_line_order).  ``line_order`` is True, False or None (the default: on for an
    orientation whose longest line exceeds four times its mean length, where lines of
    very different lengths would share wavefronts).  ``autotune`` picks the split
    threshold, the order and the batch depth per orientation by timing.  The pattern is
    validated once at construction; later calls trust it.
    """

    def __init__(self, rowptr, colidx, val, shape, *, device=None, val_dtype=torch.float32, validate=True,
                 long_len: int = DEFAULT_LONG_LEN, chunk: int = DEFAULT_CHUNK, split: bool = True,
                 line_order: Optional[bool] = None):
        device = torch.device(device or "cuda")
        if device.type != "cuda":
            raise ValueError("Pattern lives on a GPU device")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        C.load()
        self.device = device
        self.m, self.n = int(shape[0]), int(shape[1])
        self.rowptr = _dev_tensor(rowptr, torch.int32, device)
        self.colidx = _dev_tensor(colidx, torch.int32, device)
        self.val = _dev_tensor(val, val_dtype, device) if val is not None else None
        self.val_dtype = val_dtype
        self.nnz = int(self.colidx.numel())
        if self.rowptr.numel() != self.m + 1:
            raise ValueError("rowptr must have m + 1 entries")
        if self.val is not None and self.val.numel() != self.nnz:
            raise ValueError("val must have nnz entries")
        self._csr_sched = None
        self._csc_sched = None
        self._split = split
        self._orders = {C.FMM_CSR: None, C.FMM_CSC: None}
        self._hints = {C.FMM_CSR: None, C.FMM_CSC: None}  # (top, per-entry uint8 tensor)
        self._hint_cache = {}
        self._ws_cache = {}
        if validate:
            C.call("fmm_validate", ctypes.byref(self._desc(C.FMM_CSR, with_sched=False)), _stream())
        self._transpose()
        if split:
            self._csr_sched = self._schedule(self.rowptr, self.m, long_len, chunk)
            self._csc_sched = self._schedule(self.colptr, self.n, long_len, chunk)
        for o in (C.FMM_CSR, C.FMM_CSC):
            on = line_order
            if on is None:
                nl = self.m if o == C.FMM_CSR else self.n
                on = nl > 0 and self.max_line(o) > 4.0 * self.nnz / nl
            if on:
                self._orders[o] = self._order(o, self._long_len(o))
        self.csr = self._desc(C.FMM_CSR)
        self.csc = self._desc(C.FMM_CSC)

    @classmethod
    def from_csr(cls, S, **kw):
        """From any object with m, n, rowptr, colidx, val (e.g. workloads.CsrPattern)."""
        vd = torch.float64 if np.asarray(S.val).dtype == np.float64 else torch.float32
        kw.setdefault("val_dtype", vd)
        return cls(S.rowptr, S.colidx, S.val, (S.m, S.n), **kw)

    def _transpose(self):
        bytes_ = ctypes.c_size_t(0)
        C.call("fmm_csr_to_csc_workspace", self.m, self.n, self.nnz, ctypes.byref(bytes_))
        ws = torch.empty(max(1, bytes_.value), dtype=torch.uint8, device=self.device)
        self.colptr = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        self.rowidx = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        self.perm = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        self.valT = (torch.empty(self.nnz, dtype=self.val_dtype, device=self.device)
                     if self.val is not None else None)
        vcode = C.FMM_F64 if self.val_dtype == torch.float64 else C.FMM_F32
        C.call("fmm_csr_to_csc", self.m, self.n, self.nnz, _ptr(self.rowptr), _ptr(self.colidx), _ptr(self.val),
               vcode, _ptr(self.colptr), _ptr(self.rowidx), _ptr(self.valT), _ptr(self.perm), _ptr(ws),
               bytes_.value, _stream())
        torch.cuda.current_stream().synchronize()
        del ws

    def _schedule(self, ptr, nmajor, long_len, chunk):
        bytes_ = ctypes.c_size_t(0)
        C.call("fmm_schedule_workspace", nmajor, ctypes.byref(bytes_))
        ws = torch.empty(max(1, bytes_.value), dtype=torch.uint8, device=self.device)
        nch, nsp = ctypes.c_int32(0), ctypes.c_int32(0)
        C.call("fmm_schedule_count", _ptr(ptr), nmajor, long_len, chunk, ctypes.byref(nch), ctypes.byref(nsp),
               _ptr(ws), bytes_.value, _stream())
        if nsp.value == 0:
            return None
        chunks = torch.empty(3 * nch.value, dtype=torch.int32, device=self.device)
        splits = torch.empty(3 * nsp.value, dtype=torch.int32, device=self.device)
        C.call("fmm_schedule_fill", _ptr(ptr), nmajor, long_len, chunk, _ptr(chunks), _ptr(splits), _ptr(ws),
               bytes_.value, _stream())
        torch.cuda.current_stream().synchronize()
        return {"long_len": long_len, "chunk": chunk, "n_chunks": nch.value, "n_splits": nsp.value,
                "chunks": chunks, "splits": splits}

    def _order(self, orient, long_len):
        """Line processing order of one orientation (device int32 permutation)."""
        ptr, nlines = (self.rowptr, self.m) if orient == C.FMM_CSR else (self.colptr, self.n)
        order = torch.empty(max(1, nlines), dtype=torch.int32, device=self.device)
        bytes_ = ctypes.c_size_t(0)
        C.call("fmm_line_order_workspace", nlines, ctypes.byref(bytes_))
        ws = torch.empty(max(1, bytes_.value), dtype=torch.uint8, device=self.device)
        C.call("fmm_line_order", _ptr(ptr), nlines, max(1, min(long_len, _NO_SPLIT)), _ptr(order), _ptr(ws),
               bytes_.value, _stream())
        torch.cuda.current_stream().synchronize()
        return order

    def _long_len(self, orient):
        sch = self._csr_sched if orient == C.FMM_CSR else self._csc_sched
        return sch["long_len"] if sch is not None else _NO_SPLIT

    def _refresh(self, orient):
        """Rebuild one orientation's descriptor from its schedule and order, keeping the batch depth."""
        if orient == C.FMM_CSR:
            keep = self.csr.variant
            self.csr = self._desc(C.FMM_CSR)
            self.csr.variant = keep
        else:
            keep = self.csc.variant
            self.csc = self._desc(C.FMM_CSC)
            self.csc.variant = keep

    def with_values(self, s: torch.Tensor) -> "Pattern":
        """The same pattern with stored values s (nnz, CSR order, the pattern's value
        dtype): shares every index array, schedule, order and tuning; the CSC-order
        copy of s comes from the library's gather through perm."""
        if not isinstance(s, torch.Tensor) or s.dim() != 1 or s.numel() != self.nnz:
            raise ValueError(f"values must be a 1-D tensor of nnz = {self.nnz} entries")
        if s.dtype != self.val_dtype or s.device != self.device:
            raise TypeError(f"values must be {self.val_dtype} on {self.device}")
        Q = copy.copy(self)
        Q._orders = dict(self._orders)  # Q's own tuning changes must not swap tensors under self's descriptors
        Q._hints = dict(self._hints)
        Q.val = s.detach().contiguous()
        Q.valT = torch.empty(max(1, self.nnz), dtype=self.val_dtype, device=self.device)
        vcode = C.FMM_F64 if self.val_dtype == torch.float64 else C.FMM_F32
        C.call("fmm_gather_values", _ptr(self.perm), _ptr(Q.val), vcode, _ptr(Q.valT), self.nnz, _stream())
        Q.csr = Q._desc(C.FMM_CSR)
        Q.csr.variant = self.csr.variant
        Q.csc = Q._desc(C.FMM_CSC)
        Q.csc.variant = self.csc.variant
        return Q

    def set_gather_hints(self, orient, top):
        """Gather hints for one orientation (the library's fmm_gather_hints): entries whose
        minor line is among the `top` longest gather their row with the default cache
        policy, the others with the streaming policy, so the rows many entries gather stay
        in L2 and the MALL.  top None or 0 removes the hints.  Results are unchanged."""
        if not top:
            self._hints[orient] = None
        else:
            key = (orient, int(top))
            hot = self._hint_cache.get(key)
            if hot is None:
                hot = torch.empty(max(1, self.nnz), dtype=torch.uint8, device=self.device)
                minor_ptr, n_minor = (self.colptr, self.n) if orient == C.FMM_CSR else (self.rowptr, self.m)
                d = self._desc(orient)
                C.call("fmm_gather_hints", ctypes.byref(d), _ptr(minor_ptr), n_minor, int(top), _ptr(hot),
                       _stream())
                self._hint_cache[key] = hot
            self._hints[orient] = (int(top), hot)
        self._refresh(orient)

    def minor_skewed(self, orient):
        """True when the minor lines of an orientation (columns for FMM_CSR, rows for
        FMM_CSC) have hubs: the longest is over four times the mean."""
        other = C.FMM_CSC if orient == C.FMM_CSR else C.FMM_CSR
        nl = self.n if orient == C.FMM_CSR else self.m
        return nl > 0 and self.max_line(other) > 4.0 * self.nnz / nl

    @property
    def gather_hints(self):
        """Gather-hint setting of each orientation: the number of hot minor lines, or None."""
        return {k: (self._hints[o][0] if self._hints[o] is not None else None)
                for k, o in (("csr", C.FMM_CSR), ("csc", C.FMM_CSC))}

    def set_line_order(self, orient, enabled: bool):
        """Process one orientation's lines by decreasing length (True) or in index order."""
        self._orders[orient] = self._order(orient, self._long_len(orient)) if enabled else None
        self._refresh(orient)

    @property
    def orders(self):
        """Line processing order of each orientation (None when disabled)."""
        return {"csr": self._orders[C.FMM_CSR], "csc": self._orders[C.FMM_CSC]}

    def _desc(self, orient, with_sched=True):
        d = C.fmm_sparse()
        d.orient = orient
        d.rows, d.cols, d.nnz = self.m, self.n, self.nnz
        if orient == C.FMM_CSR:
            d.ptr, d.idx, d.val = self.rowptr.data_ptr(), self.colidx.data_ptr(), _ptr(self.val)
            sch = self._csr_sched
        else:
            d.ptr, d.idx, d.val = self.colptr.data_ptr(), self.rowidx.data_ptr(), _ptr(self.valT)
            d.perm = self.perm.data_ptr()
            sch = self._csc_sched
        if with_sched and sch is not None:
            d.long_len, d.n_chunks, d.n_splits = sch["long_len"], sch["n_chunks"], sch["n_splits"]
            d.chunks, d.splits = sch["chunks"].data_ptr(), sch["splits"].data_ptr()
        if with_sched and self._orders.get(orient) is not None:
            d.order = self._orders[orient].data_ptr()
        if self._hints.get(orient) is not None:
            d.hot = self._hints[orient][1].data_ptr()
        return d

    def descriptor(self, orient, schedule=True):
        """fmm_sparse descriptor for the C ABI (schedule=False drops the split schedule)."""
        if schedule:
            return self.csr if orient == C.FMM_CSR else self.csc
        return self._desc(orient, with_sched=False)

    def set_split(self, orient, long_len, chunk=None):
        """Rebuild one orientation's split schedule: lines longer than long_len are cut
        into chunks of `chunk` (default long_len) entries.  The batch depth and the
        order setting are kept."""
        chunk = chunk or long_len
        if orient == C.FMM_CSR:
            self._csr_sched = self._schedule(self.rowptr, self.m, long_len, chunk)
        else:
            self._csc_sched = self._schedule(self.colptr, self.n, long_len, chunk)
        if self._orders[orient] is not None:  # the order places split lines last
            self._orders[orient] = self._order(orient, self._long_len(orient))
        self._refresh(orient)

    def max_line(self, orient):
        """Entries in the longest line of an orientation (rows for FMM_CSR, columns for FMM_CSC)."""
        ptr = self.rowptr if orient == C.FMM_CSR else self.colptr
        return int((ptr[1:] - ptr[:-1]).max().item()) if ptr.numel() > 1 else 0

    def set_variant(self, csr=None, csc=None):
        """Batch depth class of each orientation (FMM_VARIANT_*; 0 = automatic)."""
        if csr is not None:
            self.csr.variant = int(csr)
        if csc is not None:
            self.csc.variant = int(csc)

    def launch_shape(self, orient, two_row, r, dcode):
        """(lanes, vectors per lane, elements per vector, entries per batch) of the line
        kernel a call on this orientation launches."""
        vals = [ctypes.c_int32(0) for _ in range(4)]
        C.call("fmm_launch_shape", ctypes.byref(self.descriptor(orient)), int(two_row), r, dcode,
               *[ctypes.byref(v) for v in vals])
        return tuple(v.value for v in vals)

    @property
    def variants(self):
        """Batch depth class of each orientation (FMM_VARIANT_*)."""
        return {"csr": self.csr.variant, "csc": self.csc.variant}

    def autotune(self, A, B, dC, form="a", split_candidates=SPLIT_CANDIDATES, orders=(False, True),
                 hint_candidates=True):
        """Time FusedMMA (form "a") or FusedMMB ("b") forward and adjoint on these operands
        and keep, per orientation, the fastest combination of split threshold (from
        split_candidates, where some line is longer), line order (from `orders`), gather
        hints (off, or the HINT_BYTES worth of longest minor lines, where those have hubs)
        and batch depth.  The library's fmm_autotune picks the depth for each combination;
        the forward times the orientation the forward runs on, the two-row adjoint pass
        the other one."""
        r = A.shape[1]
        dcode, odt = _common(self, A, B)
        rows_out = self.m if form == "a" else self.n
        # the library's autotuner reads dC as float32 (float64 on the F64 path); a bfloat16
        # upstream gradient is tuned with its float32 original
        _check_dense("dC", dC, rows_out, r, self.device)
        if dC.dtype != odt:
            raise TypeError(f"autotune takes dC as {odt}")
        C_out = torch.empty(rows_out, r, dtype=odt, device=self.device)
        dA = torch.empty(self.m, r, dtype=odt, device=self.device)
        dB = torch.empty(self.n, r, dtype=odt, device=self.device)
        op = C.FMM_OP_FUSEDMM_A_BWD if form == "a" else C.FMM_OP_FUSEDMM_B_BWD
        own, other = (C.FMM_CSR, C.FMM_CSC) if form == "a" else (C.FMM_CSC, C.FMM_CSR)
        if form == "a":
            def fwd():
                fusedmm_a_raw(self, A, B, out=C_out)

            def two_row():
                fusedmm_a_backward_raw(self, A, B, dC, dB=dB, need=(False, True))
        else:
            def fwd():
                fusedmm_b_raw(self, A, B, out=C_out)

            def two_row():
                fusedmm_b_backward_raw(self, A, B, dC, dA=dA, need=(True, False))

        def time_it(fn, reps=3):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        def tune_depth():
            ws, wb = self.workspace(op, r, dcode)
            C.call("fmm_autotune", op, ctypes.byref(self.csr), ctypes.byref(self.csc), _ptr(A), _ptr(B), _ptr(dC),
                   r, dcode, _ptr(C_out), _ptr(dA), _ptr(dB), _ptr(ws), wb, _stream())

        longest = max(self.max_line(C.FMM_CSR), self.max_line(C.FMM_CSC))
        cands = [ll for ll in split_candidates if ll < longest] if self._split else []
        # gather hints are tried where the gathered rows have hubs
        skewed = {o: self.minor_skewed(o) for o in (C.FMM_CSR, C.FMM_CSC)}
        top = max(1, HINT_BYTES // (r * A.element_size()))
        hints = (None, top) if hint_candidates and any(skewed.values()) else (None,)
        combos = [(lo, ll, h) for lo in orders for ll in (cands or [None]) for h in hints]
        best = {}
        for lo, ll, h in combos:
            for o in (C.FMM_CSR, C.FMM_CSC):
                if ll is not None:
                    self.set_split(o, ll)
                self.set_line_order(o, lo)
                self.set_gather_hints(o, h if skewed[o] else None)
            tune_depth()
            if len(combos) == 1:
                return self.variants
            for o, fn in ((own, fwd), (other, two_row)):
                ms = time_it(fn)
                v = self.csr.variant if o == C.FMM_CSR else self.csc.variant
                if o not in best or ms < best[o][0]:
                    best[o] = (ms, lo, ll, h if skewed[o] else None, v)
        for o, (_, lo, ll, h, v) in best.items():
            if ll is not None:
                self.set_split(o, ll)
            self.set_line_order(o, lo)
            self.set_gather_hints(o, h)
            if o == C.FMM_CSR:
                self.csr.variant = v
            else:
                self.csc.variant = v
        return self.variants

    @property
    def tuning(self):
        """Per orientation: batch depth, split threshold (None: no split schedule) and
        whether the line order is on."""
        sp = self.splits
        gh = self.gather_hints
        return {k: {"variant": (self.csr if k == "csr" else self.csc).variant, "long_len": sp[k],
                    "line_order": self.orders[k] is not None, "gather_hints": gh[k]} for k in ("csr", "csc")}

    def apply_tuning(self, tuning):
        """Put back a configuration that `tuning` reported (for instance one saved as JSON
        after `autotune` on the same pattern): per orientation the split threshold, the
        line order and the batch depth.  Results are then those of the tuned pattern, bit
        for bit."""
        for orient, key in ((C.FMM_CSR, "csr"), (C.FMM_CSC, "csc")):
            t = tuning[key]
            self.set_split(orient, t["long_len"] if t["long_len"] is not None else _NO_SPLIT)
            self.set_line_order(orient, bool(t["line_order"]))
            self.set_gather_hints(orient, t.get("gather_hints"))
        self.set_variant(tuning["csr"]["variant"], tuning["csc"]["variant"])

    @property
    def splits(self):
        """Split threshold (long_len) of each orientation's schedule, None without one."""
        return {k: (s["long_len"] if s is not None else None) for k, s in self.schedules.items()}

    @property
    def schedules(self):
        """Split schedule of each orientation (a dict of its arrays and threshold), None without one."""
        return {"csr": self._csr_sched, "csc": self._csc_sched}

    def workspace(self, op: int, r: int, dcode: int):
        """Device workspace for a call (cached by size); None when not needed."""
        bytes_ = ctypes.c_size_t(0)
        C.call("fmm_workspace_size", op, ctypes.byref(self.csr), ctypes.byref(self.csc), r, dcode,
               ctypes.byref(bytes_))
        if bytes_.value == 0:
            return None, 0
        ws = self._ws_cache.get(bytes_.value)
        if ws is None:
            ws = torch.empty(bytes_.value, dtype=torch.uint8, device=self.device)
            self._ws_cache[bytes_.value] = ws
        return ws, bytes_.value


def _common(P: Pattern, A, B):
    dcode = dtype_code(A)
    if B is not None and B.dtype != A.dtype:
        raise TypeError(f"A is {A.dtype} but B is {B.dtype}")
    want = torch.float64 if dcode == C.FMM_F64 else torch.float32
    if P.val is not None and P.val_dtype != want:
        raise TypeError(f"pattern values are {P.val_dtype}; {A.dtype} storage needs {want}")
    return dcode, _out_dtype(dcode)


# ---------------------------------------------------------------- raw calls (no autograd)

def fusedmm_a_raw(P, A, B, out=None, fused=True, R_ws=None):
    """C = FusedMMA(S, A, B) = (S * (A B^T)) B (Section II; row form in Section IV-B), no autograd.
    Fused: one pass with the sampled values in registers; unfused: SDDMM into R_ws, then
    SpMM.  Returns (C, R_ws)."""
    r = A.shape[1]
    _check_dense("A", A, P.m, r, P.device)
    _check_dense("B", B, P.n, r, P.device)
    dcode, odt = _common(P, A, B)
    out = torch.empty(P.m, r, dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, (P.m, r))
    if not fused and R_ws is None:
        R_ws = torch.empty(max(1, P.nnz), dtype=odt, device=P.device)
    elif R_ws is not None:
        _check_buf("R_ws", R_ws, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_A, r, dcode)
    C.call("fmm_fusedmm_a", ctypes.byref(P.csr), _ptr(A), _ptr(B), r, dcode, _ptr(out),
           C.FMM_FUSED if fused else C.FMM_UNFUSED, _ptr(R_ws), _ptr(ws), wb, _stream())
    return out, R_ws


def fusedmm_a_noalloc_raw(P, A, B, out):
    """C = FusedMMA(S, A, B), fused, into the caller's `out`, through the library's
    allocation-free entry point: split-line partials go to the library's own per-GPU
    array (at most NOALLOC_SCRATCH_BYTES), so the call allocates nothing, here or in the
    library.  Calls that overlap in time on one GPU race on that array."""
    r = A.shape[1]
    _check_dense("A", A, P.m, r, P.device)
    _check_dense("B", B, P.n, r, P.device)
    dcode, odt = _common(P, A, B)
    _check_buf("out", out, P.device, odt, (P.m, r))
    C.call("fmm_fusedmm_a_noalloc", ctypes.byref(P.csr), _ptr(A), _ptr(B), r, dcode, _ptr(out), _stream())
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def fusedmm_b_raw(P, A, B, out=None, fused=True, R_ws=None):
    """C' = FusedMMB(S, A, B) = (S * (A B^T))^T A, run as FusedMMA on the stored transpose with
    A and B interchanged (Section IV-B), no autograd.  Returns (C', R_ws), R_ws in CSR order."""
    r = A.shape[1]
    _check_dense("A", A, P.m, r, P.device)
    _check_dense("B", B, P.n, r, P.device)
    dcode, odt = _common(P, A, B)
    out = torch.empty(P.n, r, dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, (P.n, r))
    if not fused and R_ws is None:
        R_ws = torch.empty(max(1, P.nnz), dtype=odt, device=P.device)
    elif R_ws is not None:
        _check_buf("R_ws", R_ws, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_B, r, dcode)
    C.call("fmm_fusedmm_b", ctypes.byref(P.csc), _ptr(A), _ptr(B), r, dcode, _ptr(out),
           C.FMM_FUSED if fused else C.FMM_UNFUSED, _ptr(R_ws), _ptr(ws), wb, _stream())
    return out, R_ws


def _dc_flag(dC, dcode, odt, fused):
    """FMM_DC_BF16 when the upstream gradient is stored as bfloat16 (with bfloat16 A, B
    and the fused adjoint only), else 0; raises for any other dC dtype."""
    if dC.dtype == odt:
        return 0
    if dC.dtype == torch.bfloat16 and dcode == C.FMM_BF16:
        if not fused:
            raise ValueError("a bfloat16 dC needs the fused adjoint")
        return C.FMM_DC_BF16
    raise TypeError(f"dC must be {odt}" + (" or bfloat16" if dcode == C.FMM_BF16 else ""))


def fusedmm_a_backward_raw(P, A, B, dC, dA=None, dB=None, need=(True, True), fused=True, R_ws=None, dP_ws=None):
    """Adjoint of FusedMMA for upstream gradient dC (m x r): dA by the row pass, dB by
    the two-row column pass.  With bfloat16 A and B, dC may be bfloat16 as well (fused
    only): the passes then read it as stored."""
    r = A.shape[1]
    dcode, odt = _common(P, A, B)
    _check_dense("dC", dC, P.m, r, P.device)
    dflag = _dc_flag(dC, dcode, odt, fused)
    if need[0] and dA is None:
        dA = torch.empty(P.m, r, dtype=odt, device=P.device)
    elif need[0]:
        _check_buf("dA", dA, P.device, odt, (P.m, r))
    if need[1] and dB is None:
        dB = torch.empty(P.n, r, dtype=odt, device=P.device)
    elif need[1]:
        _check_buf("dB", dB, P.device, odt, (P.n, r))
    if not fused and dP_ws is None:
        dP_ws = torch.empty(max(1, P.nnz), dtype=odt, device=P.device)
    for name, buf in (("R_ws", R_ws), ("dP_ws", dP_ws)):
        if buf is not None:
            _check_buf(name, buf, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_A_BWD, r, dcode)
    C.call("fmm_fusedmm_a_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(A), _ptr(B), _ptr(dC), r,
           dcode, _ptr(dA if need[0] else None), _ptr(dB if need[1] else None),
           (C.FMM_FUSED if fused else C.FMM_UNFUSED) | dflag, _ptr(R_ws), _ptr(dP_ws), _ptr(ws), wb, _stream())
    return dA, dB


def fusedmm_b_backward_raw(P, A, B, dC, dA=None, dB=None, need=(True, True), fused=True, R_ws=None, dP_ws=None):
    """Adjoint of FusedMMB for upstream gradient dC (n x r); dC may be bfloat16 as for
    fusedmm_a_backward_raw."""
    r = A.shape[1]
    dcode, odt = _common(P, A, B)
    _check_dense("dC", dC, P.n, r, P.device)
    dflag = _dc_flag(dC, dcode, odt, fused)
    if need[0] and dA is None:
        dA = torch.empty(P.m, r, dtype=odt, device=P.device)
    elif need[0]:
        _check_buf("dA", dA, P.device, odt, (P.m, r))
    if need[1] and dB is None:
        dB = torch.empty(P.n, r, dtype=odt, device=P.device)
    elif need[1]:
        _check_buf("dB", dB, P.device, odt, (P.n, r))
    if not fused and dP_ws is None:
        dP_ws = torch.empty(max(1, P.nnz), dtype=odt, device=P.device)
    for name, buf in (("R_ws", R_ws), ("dP_ws", dP_ws)):
        if buf is not None:
            _check_buf(name, buf, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_B_BWD, r, dcode)
    C.call("fmm_fusedmm_b_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(A), _ptr(B), _ptr(dC), r,
           dcode, _ptr(dA if need[0] else None), _ptr(dB if need[1] else None),
           (C.FMM_FUSED if fused else C.FMM_UNFUSED) | dflag, _ptr(R_ws), _ptr(dP_ws), _ptr(ws), wb, _stream())
    return dA, dB



def fusedmm_a_backward_values_raw(P, A, B, dC, dS=None, dA=None, want_dA=False, fused=True):
    """dL/dS at S's stored entries (CSR order) for C = FusedMMA(S, A, B):
    dS_ij = <A_i, B_j> <dC_i, B_j>; with want_dA the same fused pass also gives dA."""
    r = A.shape[1]
    dcode, odt = _common(P, A, B)
    _check_dense("dC", dC, P.m, r, P.device)
    if dC.dtype != odt:
        raise TypeError(f"dC must be {odt}")
    dS = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if dS is None else \
        _check_buf("dS", dS, P.device, odt, min_numel=P.nnz)
    if want_dA and dA is None:
        dA = torch.empty(P.m, r, dtype=odt, device=P.device)
    elif want_dA:
        _check_buf("dA", dA, P.device, odt, (P.m, r))
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_A_BWD_VALUES, r, dcode)
    C.call("fmm_fusedmm_a_backward_values", ctypes.byref(P.csr), _ptr(A), _ptr(B), _ptr(dC), r, dcode, _ptr(dS),
           _ptr(dA if want_dA else None), C.FMM_FUSED if fused else C.FMM_UNFUSED, _ptr(ws), wb, _stream())
    return dS[:P.nnz], (dA if want_dA else None)


def fusedmm_b_backward_values_raw(P, A, B, dC, dS=None, dB=None, want_dB=False, fused=True):
    """dL/dS (CSR order) for C' = FusedMMB(S, A, B): dS_ij = <A_i, B_j> <A_i, dC_j>; with
    want_dB the same fused pass (on the transposed copy) also gives dB."""
    r = A.shape[1]
    dcode, odt = _common(P, A, B)
    _check_dense("dC", dC, P.n, r, P.device)
    if dC.dtype != odt:
        raise TypeError(f"dC must be {odt}")
    dS = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if dS is None else \
        _check_buf("dS", dS, P.device, odt, min_numel=P.nnz)
    if want_dB and dB is None:
        dB = torch.empty(P.n, r, dtype=odt, device=P.device)
    elif want_dB:
        _check_buf("dB", dB, P.device, odt, (P.n, r))
    ws, wb = P.workspace(C.FMM_OP_FUSEDMM_B_BWD_VALUES, r, dcode)
    C.call("fmm_fusedmm_b_backward_values", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(A), _ptr(B), _ptr(dC), r,
           dcode, _ptr(dS), _ptr(dB if want_dB else None), C.FMM_FUSED if fused else C.FMM_UNFUSED, _ptr(ws), wb,
           _stream())
    return dS[:P.nnz], (dB if want_dB else None)


def sddmm_raw(P, A, B, out=None, orient=C.FMM_CSR, beta=0.0):
    """R = S * (A B^T) at the stored entries (Eq. (1)), in CSR order (or CSC order with
    orient=FMM_CSC); out = beta out + R."""
    r = A.shape[1]
    _check_dense("A", A, P.m, r, P.device)
    _check_dense("B", B, P.n, r, P.device)
    dcode, odt = _common(P, A, B)
    out = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, min_numel=P.nnz)
    desc = P.csr if orient == C.FMM_CSR else P.csc
    C.call("fmm_sddmm", ctypes.byref(desc), _ptr(A), _ptr(B), r, dcode, _ptr(out), float(beta), None, 0, _stream())
    return out[:P.nnz]


def spmm_a_raw(P, B, w=None, out=None, beta=0.0):
    """SpMMA: out = beta out + W B, W the pattern with per-entry values w (CSR order; None =
    S's values) (Section II)."""
    r = B.shape[1]
    _check_dense("B", B, P.n, r, P.device)
    dcode, odt = _common(P, B, None)
    out = torch.empty(P.m, r, dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, (P.m, r))
    if w is not None:
        _check_buf("w", w, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_SPMM_A, r, dcode)
    C.call("fmm_spmm_a", ctypes.byref(P.csr), _ptr(w), _ptr(B), r, dcode, _ptr(out), float(beta), _ptr(ws), wb,
           _stream())
    return out


def spmm_b_raw(P, A, w=None, w_order=C.FMM_CSR, out=None, beta=0.0):
    """SpMMB: out = beta out + W^T A on the stored transpose; w in CSR order (read through
    perm) or CSC order (w_order) (Section II)."""
    r = A.shape[1]
    _check_dense("A", A, P.m, r, P.device)
    dcode, odt = _common(P, A, None)
    out = torch.empty(P.n, r, dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, (P.n, r))
    if w is not None:
        _check_buf("w", w, P.device, odt, min_numel=P.nnz)
    ws, wb = P.workspace(C.FMM_OP_SPMM_B, r, dcode)
    C.call("fmm_spmm_b", ctypes.byref(P.csc), _ptr(w), w_order, _ptr(A), r, dcode, _ptr(out), float(beta),
           _ptr(ws), wb, _stream())
    return out


# ---------------------------------------------------------------- autograd functions

def _upstream(dC, A, grad_bf16):
    """The upstream gradient as the adjoint reads it: rounded to bfloat16 storage when
    asked for (bfloat16 A and B only), else as given."""
    dC = dC.contiguous()
    if grad_bf16 and A.dtype == torch.bfloat16 and dC.dtype == torch.float32:
        return to_bf16(dC)
    return dC


class _FusedMMA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, A, B, fused, grad_bf16):
        C_out, R_ws = fusedmm_a_raw(P, A, B, fused=fused)
        ctx.P, ctx.fused, ctx.R, ctx.grad_bf16 = P, fused, R_ws, grad_bf16
        ctx.save_for_backward(A, B)
        return C_out

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        need = (ctx.needs_input_grad[1], ctx.needs_input_grad[2])
        if not any(need):
            return None, None, None, None, None
        dA, dB = fusedmm_a_backward_raw(ctx.P, A, B, _upstream(dC, A, ctx.grad_bf16), need=need, fused=ctx.fused,
                                        R_ws=ctx.R)
        return None, dA, dB, None, None


class _FusedMMB(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, A, B, fused, grad_bf16):
        C_out, R_ws = fusedmm_b_raw(P, A, B, fused=fused)
        ctx.P, ctx.fused, ctx.R, ctx.grad_bf16 = P, fused, R_ws, grad_bf16
        ctx.save_for_backward(A, B)
        return C_out

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        need = (ctx.needs_input_grad[1], ctx.needs_input_grad[2])
        if not any(need):
            return None, None, None, None, None
        dA, dB = fusedmm_b_backward_raw(ctx.P, A, B, _upstream(dC, A, ctx.grad_bf16), need=need, fused=ctx.fused,
                                        R_ws=ctx.R)
        return None, dA, dB, None, None


class _FusedMMValues(torch.autograd.Function):
    """FusedMMA / FusedMMB with S's stored values s as a differentiable input."""

    @staticmethod
    def forward(ctx, P, A, B, s, form, fused):
        Q = P.with_values(s)
        raw = fusedmm_a_raw if form == "a" else fusedmm_b_raw
        C_out, R_ws = raw(Q, A, B, fused=fused)
        ctx.Q, ctx.form, ctx.fused, ctx.R = Q, form, fused, R_ws
        ctx.save_for_backward(A, B)
        return C_out

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        Q, form, fused = ctx.Q, ctx.form, ctx.fused
        dC = dC.contiguous()
        needA, needB, needS = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        dA = dB = ds = None
        if form == "a":
            if needS:  # the fused pass that writes dS also writes dA
                ds, dA = fusedmm_a_backward_values_raw(Q, A, B, dC, want_dA=needA and fused, fused=fused)
            rest = (needA and dA is None, needB)
            if any(rest):
                xA, xB = fusedmm_a_backward_raw(Q, A, B, dC, need=rest, fused=fused, R_ws=ctx.R)
                dA = xA if rest[0] else dA
                dB = xB
        else:
            if needS:
                ds, dB = fusedmm_b_backward_values_raw(Q, A, B, dC, want_dB=needB and fused, fused=fused)
            rest = (needA, needB and dB is None)
            if any(rest):
                xA, xB = fusedmm_b_backward_raw(Q, A, B, dC, need=rest, fused=fused, R_ws=ctx.R)
                dA = xA
                dB = xB if rest[1] else dB
        return None, dA, dB, ds, None, None


class _SDDMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, A, B):
        ctx.P = P
        ctx.save_for_backward(A, B)
        return sddmm_raw(P, A, B)

    @staticmethod
    def backward(ctx, dR):
        A, B = ctx.saved_tensors
        P = ctx.P
        r = A.shape[1]
        dcode, odt = _common(P, A, B)
        dR = dR.contiguous()
        dA = torch.empty(P.m, r, dtype=odt, device=P.device) if ctx.needs_input_grad[1] else None
        dB = torch.empty(P.n, r, dtype=odt, device=P.device) if ctx.needs_input_grad[2] else None
        ws, wb = P.workspace(C.FMM_OP_SDDMM_BWD, r, dcode)
        C.call("fmm_sddmm_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(A), _ptr(B), _ptr(dR), r, dcode,
               _ptr(dA), _ptr(dB), _ptr(ws), wb, _stream())
        return None, dA, dB


class _SpMMA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, B, w):
        ctx.P = P
        ctx.save_for_backward(B, w)
        return spmm_a_raw(P, B, w)

    @staticmethod
    def backward(ctx, dC):
        B, w = ctx.saved_tensors
        P = ctx.P
        r = B.shape[1]
        dcode, odt = _common(P, B, None)
        dC = dC.contiguous()
        dB = torch.empty(P.n, r, dtype=odt, device=P.device) if ctx.needs_input_grad[1] else None
        dw = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if ctx.needs_input_grad[2] else None
        ws, wb = P.workspace(C.FMM_OP_SPMM_A_BWD, r, dcode)
        C.call("fmm_spmm_a_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(w), _ptr(B), _ptr(dC), r,
               dcode, _ptr(dw), _ptr(dB), _ptr(ws), wb, _stream())
        return None, dB, (dw[:P.nnz] if dw is not None else None)


class _SpMMB(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, A, w):
        ctx.P = P
        ctx.save_for_backward(A, w)
        return spmm_b_raw(P, A, w, C.FMM_CSR)

    @staticmethod
    def backward(ctx, dC):
        A, w = ctx.saved_tensors
        P = ctx.P
        r = A.shape[1]
        dcode, odt = _common(P, A, None)
        dC = dC.contiguous()
        dA = torch.empty(P.m, r, dtype=odt, device=P.device) if ctx.needs_input_grad[1] else None
        dw = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if ctx.needs_input_grad[2] else None
        ws, wb = P.workspace(C.FMM_OP_SPMM_B_BWD, r, dcode)
        C.call("fmm_spmm_b_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(w), _ptr(A), _ptr(dC), r,
               dcode, _ptr(dw), _ptr(dA), _ptr(ws), wb, _stream())
        return None, dA, (dw[:P.nnz] if dw is not None else None)


def fusedmm_a(P: Pattern, A, B, fused: bool = True, values: Optional[torch.Tensor] = None,
              grad_bf16: bool = False):
    """FusedMMA(S, A, B) = SpMMA(SDDMM(A, B, S), B), differentiable in A and B, and in
    S's stored values when they are given as ``values`` (nnz, CSR order).  grad_bf16
    (bfloat16 A and B, fused): the adjoint reads the upstream gradient rounded to
    bfloat16, which halves the bytes its column pass gathers for it."""
    if values is not None:
        return _FusedMMValues.apply(P, A, B, values, "a", fused)
    return _FusedMMA.apply(P, A, B, fused, grad_bf16)


def fusedmm_b(P: Pattern, A, B, fused: bool = True, values: Optional[torch.Tensor] = None,
              grad_bf16: bool = False):
    """FusedMMB(S, A, B) = SpMMB(SDDMM(A, B, S), A), differentiable in A and B, and in
    S's stored values when they are given as ``values``; grad_bf16 as for fusedmm_a."""
    if values is not None:
        return _FusedMMValues.apply(P, A, B, values, "b", fused)
    return _FusedMMB.apply(P, A, B, fused, grad_bf16)


def sddmm(P: Pattern, A, B):
    """Stored values of S * (A B^T) in CSR order (Eq. (1)), differentiable in A and B."""
    return _SDDMM.apply(P, A, B)


def spmm_a(P: Pattern, B, w=None):
    """S B, or W B where W has S's pattern and stored values w (CSR order)."""
    return _SpMMA.apply(P, B, w)


def spmm_b(P: Pattern, A, w=None):
    """S^T A, or W^T A where W has S's pattern and stored values w (CSR order)."""
    return _SpMMB.apply(P, A, w)


def gat_scores(H, a1, a2):
    """s = H a1, t = H a2 (the two halves of the attention score a^T (H_i || H_j))."""
    if not H.is_cuda or H.dim() != 2:
        raise ValueError("H must be a 2-D GPU tensor")
    n, r = H.shape
    dcode = dtype_code(H)
    odt = _out_dtype(dcode)
    if a1.dtype != odt or a2.dtype != odt:
        raise TypeError(f"attention vectors must be {odt}")
    for name, a in (("a1", a1), ("a2", a2)):
        if a.device != H.device or a.numel() != r:
            raise ValueError(f"{name} must hold r = {r} values on {H.device}")
    s = torch.empty(n, dtype=odt, device=H.device)
    t = torch.empty(n, dtype=odt, device=H.device)
    C.call("fmm_gat_scores", _ptr(H.contiguous()), n, r, dcode, _ptr(a1.contiguous()), _ptr(a2.contiguous()),
           _ptr(s), _ptr(t), _stream())
    return s, t


def gat_forward(P: Pattern, H, a1, a2, negative_slope=0.2, softmax=True, out=None, lse=None):
    """One graph-attention head (Section VI-E): out_i = sum_j w_ij H_j with
    w = LeakyReLU(S_ij (a1.H_i + a2.H_j)), row-softmaxed when ``softmax``.  With the
    softmax, ``lse`` (n values) receives each row's log-sum-exp for the adjoint."""
    if P.m != P.n:
        raise ValueError("graph attention needs a square pattern")
    r = H.shape[1]
    _check_dense("H", H, P.n, r, P.device)
    dcode, odt = _common(P, H, None)
    s, t = gat_scores(H, a1, a2)
    out = torch.empty(P.m, r, dtype=odt, device=P.device) if out is None else \
        _check_buf("out", out, P.device, odt, (P.m, r))
    nb = ctypes.c_size_t(0)
    C.call("fmm_gat_workspace", ctypes.byref(P.csr), r, dcode, ctypes.byref(nb))
    ws = None
    if nb.value:
        ws = P._ws_cache.get(("gat", nb.value))
        if ws is None:
            ws = torch.empty(nb.value, dtype=torch.uint8, device=P.device)
            P._ws_cache[("gat", nb.value)] = ws
    if lse is not None:
        _check_buf("lse", lse, P.device, odt, (P.m,))
    C.call("fmm_gat_forward", ctypes.byref(P.csr), _ptr(s), _ptr(t), _ptr(H), r, dcode, float(negative_slope),
           C.FMM_GAT_SOFTMAX if softmax else 0, _ptr(out), _ptr(lse), _ptr(ws), nb.value, _stream())
    return out


def gat_backward(P: Pattern, H, a1, a2, out, dO, negative_slope=0.2, softmax=True, want_dS=False, lse=None):
    """Adjoint of gat_forward: (dH, da1, da2, dS) for upstream gradient dO, from the
    forward's output ``out`` and, with the softmax, its ``lse`` (recomputed by a forward
    call when not given).  dS, the gradient for S's stored values in CSR order, only
    with want_dS.  With bfloat16 H, dO may be bfloat16 as well (read as stored)."""
    r = H.shape[1]
    _check_dense("H", H, P.n, r, P.device)
    dcode, odt = _common(P, H, None)
    _check_dense("out", out, P.m, r, P.device)
    if out.dtype != odt:
        raise TypeError(f"out must be {odt}")
    dO = dO.contiguous()
    _check_dense("dO", dO, P.m, r, P.device)
    if dO.dtype == odt:
        dflag = 0
    elif dO.dtype == torch.bfloat16 and dcode == C.FMM_BF16:
        dflag = C.FMM_DC_BF16
    else:
        raise TypeError(f"dO must be {odt}" + (" or bfloat16" if dcode == C.FMM_BF16 else ""))
    if lse is not None and (lse.dtype != odt or lse.numel() != P.m or not lse.is_contiguous()):
        raise ValueError(f"lse must be a contiguous {odt} vector of {P.m} values")
    if softmax and lse is None:
        lse = torch.empty(P.m, dtype=odt, device=P.device)
        gat_forward(P, H, a1, a2, negative_slope, True, out=torch.empty_like(out), lse=lse)
    s, t = gat_scores(H, a1, a2)
    dH = torch.empty(P.n, r, dtype=odt, device=P.device)
    da1 = torch.empty(r, dtype=odt, device=P.device)
    da2 = torch.empty(r, dtype=odt, device=P.device)
    dS = torch.empty(max(1, P.nnz), dtype=odt, device=P.device) if want_dS else None
    nb = ctypes.c_size_t(0)
    C.call("fmm_gat_backward_workspace", ctypes.byref(P.csr), ctypes.byref(P.csc), r, dcode, ctypes.byref(nb))
    ws = P._ws_cache.get(("gat_bwd", nb.value))
    if ws is None:
        ws = torch.empty(nb.value, dtype=torch.uint8, device=P.device)
        P._ws_cache[("gat_bwd", nb.value)] = ws
    C.call("fmm_gat_backward", ctypes.byref(P.csr), ctypes.byref(P.csc), _ptr(H), _ptr(a1.contiguous()),
           _ptr(a2.contiguous()), _ptr(s), _ptr(t), _ptr(out), _ptr(lse if softmax else None), _ptr(dO), r, dcode,
           float(negative_slope),
           (C.FMM_GAT_SOFTMAX if softmax else 0) | dflag, _ptr(dH), _ptr(da1), _ptr(da2), _ptr(dS), _ptr(ws),
           nb.value, _stream())
    return dH, da1, da2, (dS[:P.nnz] if want_dS else None)


def gat_autotune(P: Pattern, H, a1, a2, dO=None, negative_slope=0.2, softmax=True,
                 split_candidates=SPLIT_CANDIDATES, orders=(False, True), variants=(1, 2)):
    """Time the attention head (forward, plus the adjoint when dO is given) over split
    threshold x line order x batch depth, applied to both orientations, and keep the
    fastest on P.  Returns P.tuning."""
    r = H.shape[1]
    odt = _out_dtype(dtype_code(H))
    out = torch.empty(P.m, r, dtype=odt, device=P.device)
    lse = torch.empty(P.m, dtype=odt, device=P.device) if softmax else None

    def run():
        gat_forward(P, H, a1, a2, negative_slope, softmax, out=out, lse=lse)
        if dO is not None:
            gat_backward(P, H, a1, a2, out, dO, negative_slope, softmax, lse=lse)

    longest = max(P.max_line(C.FMM_CSR), P.max_line(C.FMM_CSC))
    cands = [ll for ll in split_candidates if ll < longest] if P._split else []
    best = None
    for ll in (cands or [None]):
        for lo in orders:
            for o in (C.FMM_CSR, C.FMM_CSC):
                if ll is not None:
                    P.set_split(o, ll)
                P.set_line_order(o, lo)
            for v in variants:
                P.set_variant(v, v)
                run()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    run()
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / 3
                if best is None or ms < best[0]:
                    best = (ms, ll, lo, v)
    _, ll, lo, v = best
    for o in (C.FMM_CSR, C.FMM_CSC):
        if ll is not None:
            P.set_split(o, ll)
        P.set_line_order(o, lo)
    P.set_variant(v, v)
    return P.tuning


class _GAT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, H, a1, a2, values, negative_slope, softmax, grad_bf16):
        Q = P.with_values(values) if values is not None else P
        lse = torch.empty(P.m, dtype=_out_dtype(dtype_code(H)), device=P.device) if softmax else None
        out = gat_forward(Q, H, a1, a2, negative_slope=negative_slope, softmax=softmax, lse=lse)
        ctx.Q, ctx.slope, ctx.softmax, ctx.lse, ctx.grad_bf16 = Q, negative_slope, softmax, lse, grad_bf16
        ctx.save_for_backward(H, a1, a2, out)
        return out

    @staticmethod
    def backward(ctx, dO):
        H, a1, a2, out = ctx.saved_tensors
        want_dS = ctx.needs_input_grad[4]
        dH, da1, da2, dS = gat_backward(ctx.Q, H, a1, a2, out, _upstream(dO, H, ctx.grad_bf16), ctx.slope,
                                        ctx.softmax, want_dS=want_dS, lse=ctx.lse)
        return None, dH, da1, da2, dS, None, None, None


def gat(P: Pattern, H, a1, a2, values=None, negative_slope=0.2, softmax=True, grad_bf16: bool = False):
    """The attention head as a differentiable function of H, a1, a2 and, when given,
    S's stored values (learned edge values, nnz in CSR order).  grad_bf16 (bfloat16 H):
    the adjoint reads the upstream gradient rounded to bfloat16."""
    return _GAT.apply(P, H, a1, a2, values, negative_slope, softmax, grad_bf16)


def cg_lines(P: Pattern, orient, F, rhs, lam, iters, X):
    """Batched CG on (sum_{j in line} F_j F_j^T + lam I) x = rhs for every line of the
    given orientation of P (rows for FMM_CSR, columns for FMM_CSC); X is updated in place."""
    desc = P.descriptor(orient)
    nmaj = P.m if orient == C.FMM_CSR else P.n
    r = F.shape[1]
    dcode = dtype_code(F)
    # a line gathers F at its minor indices: F has a row per column (rows as lines) or per row
    _check_dense("F", F, P.n if orient == C.FMM_CSR else P.m, r, P.device)
    _check_dense("X", X, nmaj, r, P.device)
    _check_dense("rhs", rhs, nmaj, r, P.device)
    if X.dtype != torch.float32 or rhs.dtype != torch.float32:
        raise TypeError("X and rhs are float32")
    wb = ctypes.c_size_t(0)
    C.call("fmm_cg_work_size", nmaj, r, ctypes.byref(wb))
    work = P._ws_cache.get(("cg", wb.value))
    if work is None:
        work = torch.empty(wb.value // 4, dtype=torch.float32, device=P.device)
        P._ws_cache[("cg", wb.value)] = work
    ws, wsb = P.workspace(C.FMM_OP_FUSEDMM_A if orient == C.FMM_CSR else C.FMM_OP_FUSEDMM_B, r, dcode)
    C.call("fmm_cg_lines", ctypes.byref(desc), _ptr(F), r, dcode, _ptr(rhs), float(lam), int(iters), _ptr(X),
           _ptr(work), wb.value, _ptr(ws), wsb, _stream())
    return X


def als_residual(P: Pattern, A, B):
    """sum over observed entries of (C~_ij - <A_i, B_j>)^2 (P's values are the observations),
    as a float64 device scalar."""
    r = A.shape[1]
    dcode = dtype_code(A)
    _check_dense("A", A, P.m, r, P.device)
    _check_dense("B", B, P.n, r, P.device)
    if B.dtype != A.dtype:
        raise TypeError(f"A is {A.dtype} but B is {B.dtype}")
    nb = ctypes.c_size_t(0)
    C.call("fmm_residual_workspace", ctypes.byref(P.csr), ctypes.byref(nb))
    ws = P._ws_cache.get(("res", nb.value))
    if ws is None:
        ws = torch.empty(nb.value, dtype=torch.uint8, device=P.device)
        P._ws_cache[("res", nb.value)] = ws
    out = torch.empty((), dtype=torch.float64, device=P.device)
    C.call("fmm_sddmm_residual", ctypes.byref(P.csr), _ptr(A), _ptr(B), r, dcode, _ptr(out), _ptr(ws), nb.value,
           _stream())
    return out


def als_sweep(P: Pattern, A, B, lam, cg_iters):
    """One alternating-least-squares sweep on the observed values stored in P: solve for A
    with B fixed, then for B with A fixed, each by `cg_iters` batched CG steps (the paper's
    ALS application: the CG query vectors of all rows come from one FusedMM-shaped pass)."""
    rhs_a = spmm_a_raw(P, B)  # sum_j C~_ij B_j
    cg_lines(P, C.FMM_CSR, B, rhs_a, lam, cg_iters, A)
    rhs_b = spmm_b_raw(P, A)  # sum_i C~_ij A_i
    cg_lines(P, C.FMM_CSC, A, rhs_b, lam, cg_iters, B)
    return A, B


def gat_edge_values(P: Pattern, H, a1, a2, negative_slope=0.2, softmax=True):
    """The attention edge values w (CSR order) that gat_forward applies without storing."""
    dcode, odt = _common(P, H, None)
    s, t = gat_scores(H, a1, a2)
    w = torch.empty(max(1, P.nnz), dtype=odt, device=P.device)
    C.call("fmm_gat_edge_values", ctypes.byref(P.csr), _ptr(s), _ptr(t), dcode, float(negative_slope),
           C.FMM_GAT_SOFTMAX if softmax else 0, _ptr(w), _stream())
    return w[:P.nnz]


def gat_forward_unfused(P: Pattern, H, a1, a2, negative_slope=0.2, softmax=True, out=None):
    """The unfused attention head: edge values written to memory, then an SpMM reads them."""
    w = gat_edge_values(P, H, a1, a2, negative_slope, softmax)
    return spmm_a_raw(P, H, w=w, out=out)


def to_bf16(x: torch.Tensor) -> torch.Tensor:
    """Round a float32 device tensor to bfloat16 storage with the library's kernel
    (nearest, ties to even)."""
    if x.dtype != torch.float32 or not x.is_cuda:
        raise TypeError("to_bf16 takes a float32 GPU tensor")
    x = x.contiguous()
    y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    C.call("fmm_f32_to_bf16", _ptr(x), _ptr(y), x.numel(), _stream())
    return y


def stream_copy(src: torch.Tensor, dst: torch.Tensor):
    """Streaming probe: copy src's bytes into dst with the library's plain copy kernel
    (the measured HBM ceiling for read + write traffic)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("stream_copy takes contiguous GPU tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    C.call("fmm_stream_copy", _ptr(src), _ptr(dst), nbytes, _stream())


def stream_read(src: torch.Tensor, sink: torch.Tensor, key: int = 0x9E3779B9):
    """Streaming probe: read every byte of src (the measured HBM ceiling for read-only
    traffic); sink is one int32 device word, written only if the folded value equals key."""
    if not (src.is_cuda and sink.is_cuda and src.is_contiguous()) or sink.dtype != torch.int32 or sink.numel() < 1:
        raise ValueError("stream_read takes a contiguous GPU tensor and a one-word int32 GPU sink")
    C.call("fmm_stream_read", _ptr(src), src.numel() * src.element_size(), key, _ptr(sink), _stream())

def stream_gather(src: torch.Tensor, row_bytes: int, rows: torch.Tensor, sink: torch.Tensor,
                  key: int = 0x9E3779B9):
    """Gather probe: read the rows `rows` (int32 device tensor) of src viewed as rows of
    row_bytes bytes (16 * 2^k, k <= 6), one 16-byte load per lane, as the line kernels
    gather; sink as for stream_read.  Every index is checked against src's row count here,
    before the launch."""
    if not (src.is_cuda and rows.is_cuda and sink.is_cuda and src.is_contiguous() and rows.is_contiguous()):
        raise ValueError("stream_gather takes contiguous GPU tensors")
    if rows.dtype != torch.int32 or sink.dtype != torch.int32 or sink.numel() < 1:
        raise ValueError("rows must be int32 and sink one int32 word")
    nbytes = src.numel() * src.element_size()
    if row_bytes < 16 or row_bytes > 1024 or row_bytes & (row_bytes - 1) or nbytes % row_bytes:
        raise ValueError("row_bytes must be 16 * 2^k (k <= 6) and divide src's size")
    if rows.numel() and (int(rows.min()) < 0 or int(rows.max()) >= nbytes // row_bytes):
        raise ValueError("a row index lies outside src")
    C.call("fmm_stream_gather", _ptr(src), row_bytes, _ptr(rows), rows.numel(), key, _ptr(sink), _stream())


def set_tuning(lanes: int = 0, nv: int = 0):
    """Force the lane-group shape of later launches ((0, 0) = automatic)."""
    C.call("fmm_set_tuning", lanes, nv)


def device_info():
    """Compute units and architecture name of the current device."""
    cu = ctypes.c_int32(0)
    buf = ctypes.create_string_buffer(64)
    C.call("fmm_device_info", ctypes.byref(cu), buf, 64)
    return {"num_cu": cu.value, "arch": buf.value.decode()}


class BatchPlan:
    """Fused FusedMMA forward and/or adjoint over many graphs in one persistent launch.

    ``patterns[g]``, ``A[g]`` (rows x r), ``B[g]`` (cols x r) and, for the adjoint,
    ``dC[g]`` (rows x r float32; bfloat16 too when A and B are bfloat16, the same for
    every graph) describe graph g.  Outputs ``C``, ``dA``, ``dB`` are
    allocated here (lists of float32 tensors).  ``autotune()`` picks the schedule,
    ``run()`` launches eagerly, ``capture(stream)`` records the launch in a hipGraph
    and ``launch(stream)`` replays it.
    """

    def __init__(self, patterns, A, B, dC=None, forward=True, backward=True):
        if not patterns:
            raise ValueError("empty batch")
        if backward and dC is None:
            raise ValueError("the adjoint needs dC")
        self.patterns, self.A, self.B, self.dC = list(patterns), list(A), list(B), dC
        dev = patterns[0].device
        r = A[0].shape[1]
        dcode = dtype_code(A[0])
        self.r, self.dcode = r, dcode
        flags = (C.FMM_BATCH_FWD if forward else 0) | (C.FMM_BATCH_BWD if backward else 0)
        dc_dtype = dC[0].dtype if backward else torch.float32
        if dc_dtype == torch.bfloat16 and dcode == C.FMM_BF16:
            flags |= C.FMM_BATCH_DC_BF16
        elif dc_dtype != torch.float32:
            raise TypeError("dC must be float32" + (" or bfloat16" if dcode == C.FMM_BF16 else ""))
        # every graph is checked before anything is allocated or any library call is made
        for g, P in enumerate(patterns):
            if P.device != dev:
                raise ValueError(f"graph {g}'s pattern is on {P.device}, graph 0's on {dev}")
            _check_dense("A", A[g], P.m, r, dev)
            _check_dense("B", B[g], P.n, r, dev)
            if A[g].dtype != A[0].dtype or B[g].dtype != A[0].dtype:
                raise TypeError("all graphs need the same storage dtype")
            _common(P, A[g], B[g])  # the kernel reads stored values as float32
            if backward:
                _check_dense("dC", dC[g], P.m, r, dev)
                if dC[g].dtype != dc_dtype:
                    raise TypeError("every graph's dC needs the same dtype")
        self.C = [torch.empty(P.m, r, dtype=torch.float32, device=dev) for P in patterns] if forward else None
        self.dA = [torch.empty(P.m, r, dtype=torch.float32, device=dev) for P in patterns] if backward else None
        self.dB = [torch.empty(P.n, r, dtype=torch.float32, device=dev) for P in patterns] if backward else None
        arr = (C.fmm_batch_graph * len(patterns))()
        for g, P in enumerate(patterns):
            x = arr[g]
            x.csr = P.descriptor(C.FMM_CSR, schedule=False)
            x.csc = P.descriptor(C.FMM_CSC, schedule=False)
            x.A, x.B = A[g].data_ptr(), B[g].data_ptr()
            if backward:
                x.dC, x.dA, x.dB = dC[g].data_ptr(), self.dA[g].data_ptr(), self.dB[g].data_ptr()
            if forward:
                x.C = self.C[g].data_ptr()
        self._arr = arr
        self._plan = ctypes.c_void_p()
        C.call("fmm_batch_plan_create", arr, len(patterns), r, dcode, flags, ctypes.byref(self._plan))

    def autotune(self, stream=None):
        """Time every candidate schedule and keep the fastest (synchronous); returns info()."""
        C.call("fmm_batch_autotune", self._plan, self._s(stream))
        return self.info()

    PLACE_GLOBAL, PLACE_XCD, PLACE_QUEUES = 0, 1, 2

    def set_schedule(self, tile_nnz=8192, placement=PLACE_XCD, row_wave=False, col_wave=False):
        """Choose the schedule by hand: tile size, placement (PLACE_GLOBAL: LPT over all
        workgroups; PLACE_XCD: graphs pinned to XCDs, fixed lists; PLACE_QUEUES: graphs
        pinned to XCDs, tiles claimed in order from a queue per XCD; a bool means XCD or
        global), and the wavefront-per-line schedule for the row passes and for the
        column pass."""
        C.call("fmm_batch_set_schedule", self._plan, tile_nnz, int(placement), int(row_wave), int(col_wave))

    def run(self, stream=None):
        """One eager persistent launch of the current schedule."""
        C.call("fmm_batch_run", self._plan, self._s(stream))

    def capture(self, stream):
        """Record the launch in a hipGraph on `stream` (a created, non-default stream)."""
        C.call("fmm_batch_capture", self._plan, self._s(stream))

    def launch(self, stream):
        """Replay the captured hipGraph on `stream`."""
        C.call("fmm_batch_launch", self._plan, self._s(stream))

    def info(self):
        """The current schedule, its tile count and the last autotune's record."""
        i = C.fmm_batch_info()
        C.call("fmm_batch_plan_info", self._plan, ctypes.byref(i))
        return {f: getattr(i, f) for f, _ in C.fmm_batch_info._fields_}

    @staticmethod
    def _s(stream):
        if stream is None:
            return _stream()
        return ctypes.c_void_p(stream.cuda_stream)

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan:
            try:
                C.load().fmm_batch_plan_destroy(plan)
            except Exception:
                pass
            self._plan = None
