"""MI355X (gfx950) sparse matrix-matrix product C = A * B on FP64 CSR.

Python binding of the HIP library in ``csrc/`` (C ABI: ``include/spgemm.h``).
PyTorch only provides device memory and the stream; every step of the product
runs in the library's kernels.  The functions below allocate the workspace,
scratch and output tensors that the C calls ask for and pass raw pointers.

The product follows the paper's row-major (Gustavson) algorithm, Section IV-A
of Scharpff, Iglberger, Hager and Ruede (arXiv:1303.1651), with output rows
sorted by column (Section IV-B) and sizes bounded by the multiplication count
(Section IV-B).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import (OPT_FAST, OPT_VALIDATE, SIZER_EXACT, SIZER_LEARNED, SIZER_UPPER_BOUND,
                   SpgemmError, check)

SIZERS = {"exact": SIZER_EXACT, "upper_bound": SIZER_UPPER_BOUND, "learned": SIZER_LEARNED}


@dataclass
class DeviceCSR:
    rows: int
    cols: int
    row_ptr: torch.Tensor   # int64, rows + 1
    col: torch.Tensor       # int32
    val: torch.Tensor       # float64

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, M, device="cuda") -> "DeviceCSR":
        return cls(int(M.rows), int(M.cols),
                   torch.as_tensor(np.ascontiguousarray(M.row_ptr, dtype=np.int64)).to(device),
                   torch.as_tensor(np.ascontiguousarray(M.col, dtype=np.int32)).to(device),
                   torch.as_tensor(np.ascontiguousarray(M.val, dtype=np.float64)).to(device))

    def descriptor(self) -> _lib.spgemm_csr:
        return _lib.spgemm_csr(self.rows, self.cols, self.nnz, self.row_ptr.data_ptr(),
                               self.col.data_ptr() if self.nnz else None,
                               self.val.data_ptr() if self.nnz else None)

    def to_host(self):
        from types import SimpleNamespace
        return SimpleNamespace(rows=self.rows, cols=self.cols, row_ptr=self.row_ptr.cpu().numpy(),
                               col=self.col.cpu().numpy(), val=self.val.cpu().numpy())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def make_tuning(**kw) -> _lib.spgemm_tuning:
    t = _lib.spgemm_tuning()
    names = {f for f, _ in t._fields_}
    for k, v in kw.items():
        if k not in names:
            raise KeyError("unknown tuning field %r (fields: %s)" % (k, ", ".join(sorted(names))))
        setattr(t, k, v)
    return t


class Model:
    """Learned row-size network (host object in the library)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    @classmethod
    def create(cls, theta, mu, sd) -> "Model":
        th = np.ascontiguousarray(theta, dtype=np.float32)
        m = np.ascontiguousarray(mu, dtype=np.float32)
        s = np.ascontiguousarray(sd, dtype=np.float32)
        assert th.size == _lib.MLP_PARAMS and m.size == 3 and s.size == 3
        h = ctypes.c_void_p()
        check(_lib.spgemm_model_create(_f32p(th), _f32p(m), _f32p(s), ctypes.byref(h)), "spgemm_model_create")
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "Model":
        h = ctypes.c_void_p()
        check(_lib.spgemm_model_load(path.encode(), ctypes.byref(h)), "spgemm_model_load")
        return cls(h.value)

    def save(self, path: str):
        check(_lib.spgemm_model_save(self.handle, path.encode()), "spgemm_model_save")

    def params(self):
        th = np.zeros(_lib.MLP_PARAMS, np.float32)
        mu = np.zeros(3, np.float32)
        sd = np.zeros(3, np.float32)
        check(_lib.spgemm_model_get(self.handle, _f32p(th), _f32p(mu), _f32p(sd)), "spgemm_model_get")
        return th, mu, sd

    def predict(self, f1, f2, f3, stream=None) -> torch.Tensor:
        n = int(f1.numel())
        out = torch.empty(n, dtype=torch.float32, device=f1.device)
        dev = _bytes(_lib.spgemm_model_device_bytes(), f1.device)
        check(_lib.spgemm_model_predict(self.handle, f1.data_ptr(), f2.data_ptr(), f3.data_ptr(), n,
                                        out.data_ptr(), dev.data_ptr(), _stream_ptr(stream)),
              "spgemm_model_predict")
        return out

    def loss_grad(self, f1, f2, f3, nnz_c, stream=None):
        n = int(f1.numel())
        grad = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=f1.device)
        scratch = _bytes(_lib.spgemm_model_grad_scratch(n), f1.device)
        loss = ctypes.c_float()
        check(_lib.spgemm_model_loss_grad(self.handle, f1.data_ptr(), f2.data_ptr(), f3.data_ptr(),
                                          nnz_c.data_ptr(), n, grad.data_ptr(), scratch.data_ptr(),
                                          ctypes.byref(loss), _stream_ptr(stream)), "spgemm_model_loss_grad")
        return float(loss.value), grad

    def __del__(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            try:
                _lib.spgemm_model_destroy(self.handle)
            except (AttributeError, TypeError):   # interpreter shutdown: module globals already cleared
                pass
            self.handle = None


def _f32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def row_features(A: DeviceCSR, B: DeviceCSR, stream=None):
    """(nnz(A_i), multiplication count, longest selected B row) per row, int32 on the device."""
    n = A.rows
    f1 = torch.empty(n, dtype=torch.int32, device=A.row_ptr.device)
    f2 = torch.empty_like(f1)
    f3 = torch.empty_like(f1)
    da, db = A.descriptor(), B.descriptor()
    check(_lib.spgemm_row_features(ctypes.byref(da), ctypes.byref(db), f1.data_ptr(), f2.data_ptr(),
                                   f3.data_ptr(), _stream_ptr(stream)), "spgemm_row_features")
    return f1, f2, f3


def feature_stats(f1, f2, f3, stream=None):
    n = int(f1.numel())
    scratch = _bytes(_lib.spgemm_model_stats_scratch(n), f1.device)
    mu = np.zeros(3, np.float32)
    sd = np.zeros(3, np.float32)
    check(_lib.spgemm_model_feature_stats(f1.data_ptr(), f2.data_ptr(), f3.data_ptr(), n, _f32p(mu), _f32p(sd),
                                          scratch.data_ptr(), _stream_ptr(stream)), "spgemm_model_feature_stats")
    return mu, sd


def train_model(theta0, mu, sd, f1, f2, f3, nnz_c, epochs=30, batch_size=65536, lr=3e-3,
                beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """Trains the network on the device with the library's kernels."""
    n = int(f1.numel())
    hp = _lib.spgemm_train_params(epochs, batch_size, lr, beta1, beta2, eps)
    scratch = _bytes(_lib.spgemm_model_train_scratch(n, batch_size), f1.device)
    th = np.ascontiguousarray(theta0, dtype=np.float32)
    m = np.ascontiguousarray(mu, dtype=np.float32)
    s = np.ascontiguousarray(sd, dtype=np.float32)
    curve = np.zeros(epochs, np.float32)
    h = ctypes.c_void_p()
    check(_lib.spgemm_model_train(_f32p(th), _f32p(m), _f32p(s), f1.data_ptr(), f2.data_ptr(), f3.data_ptr(),
                                  nnz_c.data_ptr(), n, ctypes.byref(hp), scratch.data_ptr(), scratch.numel(),
                                  _f32p(curve), ctypes.byref(h), _stream_ptr(stream)), "spgemm_model_train")
    return Model(h.value), curve


def fit_model(pairs, seed=1001, per_source=None, epochs=30, batch_size=8192, lr=3e-3, theta0=None):
    """Trains the row-size network on the device from products (A, B) of
    DeviceCSR operands: features from the library's feature kernel, labels
    (exact nnz(C_i)) from its symbolic pass.  ``per_source`` rows are drawn
    from each source with replacement (a seeded generator), so that every
    source weighs the same; None takes every row of every source.  Rows are
    shuffled once, then trained in mini-batches by the library's kernels.
    ``theta0``: starting parameters (1,217 floats), or None for a He-uniform
    start drawn with ``seed``.  Returns (model, facts)."""
    feats, labels = [], []
    for dA, dB in pairs:
        f1, f2, f3 = row_features(dA, dB)
        plan = Plan(dA, dB, "exact")
        rp, _ = plan.symbolic()
        plan.close()
        feats.append((f1, f2, f3))
        labels.append((rp[1:] - rp[:-1]).to(torch.int32))
        del rp
    g = torch.Generator(device="cpu").manual_seed(seed)
    if per_source is None:
        picks = [None] * len(feats)
    else:
        picks = [torch.randint(0, f[0].numel(), (per_source,), generator=g).to(f[0].device) for f in feats]
    take = lambda x, i: x if i is None else x[i]
    f1 = torch.cat([take(f[0], i) for f, i in zip(feats, picks)])
    f2 = torch.cat([take(f[1], i) for f, i in zip(feats, picks)])
    f3 = torch.cat([take(f[2], i) for f, i in zip(feats, picks)])
    lab = torch.cat([take(l, i) for l, i in zip(labels, picks)])
    del feats, labels
    perm = torch.randperm(f1.numel(), generator=g).to(f1.device)
    f1, f2, f3, lab = f1[perm].contiguous(), f2[perm].contiguous(), f3[perm].contiguous(), lab[perm].contiguous()
    mu, sd = feature_stats(f1, f2, f3)
    if theta0 is None:
        theta0 = _he_uniform(seed)
    model, curve = train_model(theta0, mu, sd, f1, f2, f3, lab, epochs=epochs, batch_size=batch_size, lr=lr)
    return model, {"train_rows": int(f1.numel()), "loss_first": float(curve[0]), "loss_last": float(curve[-1])}


def _he_uniform(seed, hidden=32):
    """Start of the 3-32-32-1 network: weights uniform in +-sqrt(6 / fan_in)
    (He et al., 2015, uniform form) from a seeded generator, biases zero."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, hidden * 3) * np.sqrt(6.0 / 3.0)
    w2 = rng.uniform(-1, 1, hidden * hidden) * np.sqrt(6.0 / hidden)
    w3 = rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden)
    z = np.zeros(hidden)
    return np.concatenate([w1, z, w2, z, w3, [0.0]]).astype(np.float32)


@dataclass
class Result:
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    info: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.info.get("c_nnz", self.col.numel()))


class Plan:
    """One product C = A * B: plan, then (symbolic) and numeric passes."""

    def __init__(self, A: DeviceCSR, B: DeviceCSR, sizer="exact", model: Model | None = None,
                 fast=False, validate=False, tuning: dict | None = None, stream=None, timing=False,
                 alloc_scratch=True):
        self.A, self.B = A, B
        self.device = A.row_ptr.device
        self.stream = stream
        self._da, self._db = A.descriptor(), B.descriptor()
        self._tuning = make_tuning(**tuning) if tuning else None
        flags = (OPT_FAST if fast else 0) | (OPT_VALIDATE if validate else 0) | (_lib.OPT_TIMING if timing else 0)
        self._opts = _lib.spgemm_options(SIZERS[sizer] if isinstance(sizer, str) else int(sizer), flags,
                                         model.handle if model is not None else None,
                                         ctypes.pointer(self._tuning) if self._tuning is not None else None)
        self.model = model
        nbytes = _lib.SZ()
        check(_lib.spgemm_plan_workspace_size(ctypes.byref(self._da), ctypes.byref(self._db),
                                              ctypes.byref(self._opts), ctypes.byref(nbytes)),
              "spgemm_plan_workspace_size")
        self.workspace = _bytes(nbytes.value, self.device)
        self.handle = ctypes.c_void_p()
        info = _lib.spgemm_info()
        code = _lib.spgemm_plan_create(ctypes.byref(self._da), ctypes.byref(self._db), ctypes.byref(self._opts),
                                       self.workspace.data_ptr(), self.workspace.numel(), _stream_ptr(stream),
                                       ctypes.byref(self.handle), ctypes.byref(info))
        check(code, "spgemm_plan_create")
        self.info = info.as_dict()
        # alloc_scratch=False: the caller sets .scratch (say, one buffer that
        # plans used one after another share)
        self.scratch = (_bytes(self.info["scratch_bytes"], self.device)
                        if alloc_scratch and self.info["scratch_bytes"] else None)

    def _scratch(self):
        return (self.scratch.data_ptr(), self.scratch.numel()) if self.scratch is not None else (None, 0)

    def refresh_info(self) -> dict:
        info = _lib.spgemm_info()
        check(_lib.spgemm_plan_info(self.handle, ctypes.byref(info)), "spgemm_plan_info")
        self.info = info.as_dict()
        return self.info

    def symbolic(self, c_row_ptr: torch.Tensor | None = None):
        if c_row_ptr is None:
            c_row_ptr = torch.empty(self.A.rows + 1, dtype=torch.int64, device=self.device)
        nnz = ctypes.c_int64()
        sp, sb = self._scratch()
        code = _lib.spgemm_symbolic(self.handle, sp, sb, c_row_ptr.data_ptr(), ctypes.byref(nnz),
                                    _stream_ptr(self.stream))
        check(code, "spgemm_symbolic")
        self.refresh_info()
        return c_row_ptr, int(nnz.value)

    def numeric(self, c_row_ptr, c_col, c_val, capacity=None):
        cap = c_col.numel() if capacity is None else capacity
        nnz = ctypes.c_int64()
        sp, sb = self._scratch()
        code = _lib.spgemm_numeric(self.handle, sp, sb, None, None, c_row_ptr.data_ptr(),
                                   c_col.data_ptr() if c_col.numel() else None,
                                   c_val.data_ptr() if c_val.numel() else None, cap, ctypes.byref(nnz),
                                   _stream_ptr(self.stream))
        self.refresh_info()
        return code, int(nnz.value)

    def compute_only(self):
        """Accumulates every row of C without storing it (the pure
        computation kernel of Section IV-A); returns each row's entry count
        (int32) and largest |value| (float64) as device tensors."""
        n = self.A.rows
        cnt = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        mx = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        check(_lib.spgemm_compute_only(self.handle, None, None, cnt.data_ptr(), mx.data_ptr(),
                                       _stream_ptr(self.stream)), "spgemm_compute_only")
        self.refresh_info()
        return cnt[:n], mx[:n]

    def numeric_static(self, c_row_ptr, c_col, c_val, capacity=None):
        """The numeric pass with the library's static scratch (no allocation
        by the library; the outputs are the caller's)."""
        cap = c_col.numel() if capacity is None else capacity
        nnz = ctypes.c_int64()
        code = _lib.spgemm_numeric_static(self.handle, None, None, c_row_ptr.data_ptr(),
                                          c_col.data_ptr() if c_col.numel() else None,
                                          c_val.data_ptr() if c_val.numel() else None, cap, ctypes.byref(nnz),
                                          _stream_ptr(self.stream))
        self.refresh_info()
        return code, int(nnz.value)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.spgemm_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):   # interpreter shutdown: module globals already cleared
            pass


def spgemm(A: DeviceCSR, B: DeviceCSR, sizer="exact", model: Model | None = None, fast=False,
           validate=False, tuning: dict | None = None, stream=None) -> Result:
    """C = A * B.  ``sizer``: "exact" (symbolic + numeric), "upper_bound" or
    "learned" (one pass: rows laid out by their capacities, then compacted)."""
    plan = Plan(A, B, sizer, model, fast, validate, tuning, stream)
    try:
        dev = plan.device
        if plan.info is not None and (SIZERS[sizer] if isinstance(sizer, str) else sizer) == SIZER_EXACT:
            rp, nnz = plan.symbolic()
            col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
            val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
            code, got = plan.numeric(rp, col, val, capacity=nnz)
            check(code, "spgemm_numeric")
        else:
            rp = torch.empty(A.rows + 1, dtype=torch.int64, device=dev)
            cap = max(int(plan.info["c_capacity_hint"]), 1)
            col = torch.empty(cap, dtype=torch.int32, device=dev)
            val = torch.empty(cap, dtype=torch.float64, device=dev)
            code, got = plan.numeric(rp, col, val, capacity=cap)
            if code == 6:   # SPGEMM_E_CAPACITY: grow to the reported size and run again
                col = torch.empty(max(got, 1), dtype=torch.int32, device=dev)
                val = torch.empty(max(got, 1), dtype=torch.float64, device=dev)
                code, got = plan.numeric(rp, col, val, capacity=got)
            check(code, "spgemm_numeric")
        info = dict(plan.info)
        return Result(rp, col[:got], val[:got], info)
    finally:
        plan.close()


def transpose(M: DeviceCSR, values=True, stream=None) -> DeviceCSR:
    """The CSR of M^T, by the library's transpose kernels.  A matrix stored by
    columns (CSC) has the arrays of the CSR of its transpose, so
    ``transpose(B_csc)`` gives B by rows (the conversion Section IV-A applies
    to a right-hand operand stored by columns).  ``values=False`` moves the
    structure only (the values of the result are then unset)."""
    dev = M.row_ptr.device
    t_rp = torch.empty(M.cols + 1, dtype=torch.int64, device=dev)
    t_col = torch.empty(max(M.nnz, 1), dtype=torch.int32, device=dev)
    t_val = torch.empty(max(M.nnz, 1), dtype=torch.float64, device=dev)
    d = M.descriptor()
    scratch = _bytes(_lib.spgemm_transpose_scratch(ctypes.byref(d)), dev)
    check(_lib.spgemm_transpose(ctypes.byref(d), t_rp.data_ptr(), t_col.data_ptr(),
                                t_val.data_ptr() if values else None, scratch.data_ptr(), scratch.numel(),
                                _stream_ptr(stream)), "spgemm_transpose")
    return DeviceCSR(M.cols, M.rows, t_rp, t_col[:M.nnz], t_val[:M.nnz])


def spgemm_csc(A: DeviceCSR, B_csc: DeviceCSR, sizer="exact", **kw) -> Result:
    """C = A * B with B stored by columns: ``B_csc`` holds B's CSC arrays as
    the CSR of B^T (rows = B.cols).  B is converted to rows first, then the
    row-major product runs (Section IV-A)."""
    return spgemm(A, transpose(B_csc, stream=kw.get("stream")), sizer=sizer, **kw)


class Batch:
    """Many independent products C_i = A_i * B_i in one plan and one
    persistent launch (graph-replayed after the first run).  Argument
    marshalling only: every step runs in the library."""

    def __init__(self, As, Bs, sizer="upper_bound", model: Model | None = None, tuning: dict | None = None,
                 stream=None, timing=False):
        assert len(As) == len(Bs)
        self.As, self.Bs = list(As), list(Bs)
        self.count = len(self.As)
        self.stream = stream
        self.device = self.As[0].row_ptr.device if self.count else torch.device("cuda")
        self._da = (_lib.spgemm_csr * max(self.count, 1))(*[a.descriptor() for a in self.As])
        self._db = (_lib.spgemm_csr * max(self.count, 1))(*[b.descriptor() for b in self.Bs])
        self._tuning = make_tuning(**tuning) if tuning else None
        flags = _lib.OPT_TIMING if timing else 0
        self._opts = _lib.spgemm_options(SIZERS[sizer] if isinstance(sizer, str) else int(sizer), flags,
                                         model.handle if model is not None else None,
                                         ctypes.pointer(self._tuning) if self._tuning is not None else None)
        self.row_base = np.zeros(self.count + 1, dtype=np.int64)
        ws = _lib.SZ()
        self.handle = ctypes.c_void_p()
        check(_lib.spgemm_batched_plan(self.count, self._da, self._db, ctypes.byref(self._opts),
                                       self.row_base.ctypes.data_as(_lib.I64_P), ctypes.byref(ws),
                                       ctypes.byref(self.handle)), "spgemm_batched_plan")
        self.workspace = _bytes(ws.value, self.device)
        cap, sb = ctypes.c_int64(), _lib.SZ()
        check(_lib.spgemm_batched_reserve(self.handle, self.workspace.data_ptr(), self.workspace.numel(),
                                          ctypes.byref(cap), ctypes.byref(sb), _stream_ptr(stream)),
              "spgemm_batched_reserve")
        self.capacity = int(cap.value)
        self.scratch = _bytes(sb.value, self.device) if sb.value else None
        self.row_pool = torch.empty(int(self.row_base[-1]), dtype=torch.int64, device=self.device)
        self.col_pool = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
        self.val_pool = torch.empty(max(self.capacity, 1), dtype=torch.float64, device=self.device)

    def uses_graph(self) -> bool:
        return bool(_lib.spgemm_batched_uses_graph(self.handle))

    def run(self):
        """Runs every product; returns (nnz_base, nnz) as host arrays."""
        base = np.zeros(self.count + 1, dtype=np.int64)
        nnz = np.zeros(max(self.count, 1), dtype=np.int64)
        req = ctypes.c_int64()
        sp = self.scratch.data_ptr() if self.scratch is not None else None
        sb = self.scratch.numel() if self.scratch is not None else 0
        for _ in range(2):
            code = _lib.spgemm_batched(self.handle, sp, sb, self.row_pool.data_ptr(), self.col_pool.data_ptr(),
                                       self.val_pool.data_ptr(), self.capacity,
                                       base.ctypes.data_as(_lib.I64_P), nnz.ctypes.data_as(_lib.I64_P),
                                       ctypes.byref(req), _stream_ptr(self.stream))
            if code == 6:   # pools too small (learned capacities): grow and run again
                self.capacity = int(req.value)
                self.col_pool = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
                self.val_pool = torch.empty(max(self.capacity, 1), dtype=torch.float64, device=self.device)
                continue
            check(code, "spgemm_batched")
            break
        self.nnz_base, self.nnz = base, nnz[:self.count]
        return self.nnz_base, self.nnz

    def product(self, i: int):
        """Host copy (row_ptr, col, val) of product i after run()."""
        rp = self.row_pool[int(self.row_base[i]):int(self.row_base[i + 1])].cpu().numpy()
        b, n = int(self.nnz_base[i]), int(self.nnz[i])
        return rp, self.col_pool[b:b + n].cpu().numpy(), self.val_pool[b:b + n].cpu().numpy()

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.spgemm_batched_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):   # interpreter shutdown: module globals already cleared
            pass
