"""Thin Python binding of libclomp.so (ctypes): argument marshalling only.

Every step of the solve runs in the library's HIP kernels.  torch supplies
device memory and the stream; there is no CPU or PyTorch fallback: if the
library has not been built, or no GPU is present, calls raise.

Storage convention: a measurement matrix A (m x n) is passed atom-major as a
tensor `At` of shape (n, lda) -- row j holds column a_j -- which is A stored
column-major with leading dimension lda >= m.
"""

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclomp.so")

F32, BF16, F64 = 0, 1, 2
METHOD_CLOMP, METHOD_OMP, METHOD_IHT, METHOD_PAPER = 0, 1, 2, 3
METHODS = {"clomp": METHOD_CLOMP, "omp": METHOD_OMP, "iht": METHOD_IHT,
           "clomp_paper": METHOD_PAPER}
ST_NAN, ST_K_CAPPED, ST_ZERO_Y, ST_REFINE_INACCURATE, ST_WATCHDOG = 1, 2, 4, 8, 32
FLAG_GRAPH, FLAG_NO_FUSED_SMALL, FLAG_AUTOTUNE, FLAG_PROFILE = 1, 2, 4, 8
FLAG_RESIDUAL_FLOW, FLAG_CORR_FLOW, FLAG_NO_SHARED_GRAM, FLAG_NO_REFINE = 16, 32, 64, 128
FLAG_IMAGE = 256
PHASES = ("scan", "gram", "coef", "resid", "refine", "norm", "init", "pass", "fused")

STATUS_NAMES = {0: "CLOMP_OK", 1: "CLOMP_INVALID_ARGUMENT", 2: "CLOMP_OUT_OF_MEMORY",
                3: "CLOMP_DEVICE_ERROR", 4: "CLOMP_NOT_SUPPORTED"}


class Params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("inner_steps", ctypes.c_int32),
                ("lr_rel", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps_rel", ctypes.c_float),
                ("resid_tol", ctypes.c_float), ("refine_iters", ctypes.c_int32),
                ("refine_tol", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("select_threshold", ctypes.c_float), ("prior_tv", ctypes.c_float),
                ("prior_lv", ctypes.c_float)]


class Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lda", ctypes.c_int64),
                ("lda_master", ctypes.c_int64), ("A", ctypes.c_void_p),
                ("A_master", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("support", ctypes.c_void_p),
                ("n_selected", ctypes.c_void_p), ("resid_norm", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


# numpy view of clomp_instance_t, for packing large batches without a
# per-field ctypes assignment
INSTANCE_NP = np.dtype([(name, np.int32 if ct is ctypes.c_int32 else
                         np.int64 if ct is ctypes.c_int64 else np.uint64)
                        for name, ct in Instance._fields_])
assert INSTANCE_NP.itemsize == ctypes.sizeof(Instance)


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 12), ("launches", ctypes.c_int64 * 12),
                ("scan_bytes", ctypes.c_double), ("pass_bytes", ctypes.c_double),
                ("fused_bytes", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("scan_tile_kb", ctypes.c_int32), ("pass_tile_kb", ctypes.c_int32),
                ("team_min_rows", ctypes.c_int32), ("rscan_min_t", ctypes.c_int32),
                ("shared_min_tiles", ctypes.c_int32), ("spin_limit", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


@dataclass
class PreparedBatch:
    arr: np.ndarray          # packed clomp_instance_t descriptors
    count: int
    dtype: int
    result: "BatchResult"
    items: list              # inputs, kept alive with the batch
    stream: object
    outputs: tuple
    recorded: set = field(default_factory=set)   # streams the tensors are recorded on


class ClompError(RuntimeError):
    pass


_lib = None


def load_library(path=LIB_PATH):
    """Open libclomp.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ClompError(f"{path} is missing: build it with "
                         "`python -m paper_2501_11592_amd.build`")
    lib = ctypes.CDLL(path)
    H = ctypes.c_void_p
    lib.clomp_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.clomp_default_params.restype = None
    lib.clomp_create.argtypes = [ctypes.POINTER(H), ctypes.c_int, ctypes.POINTER(Params)]
    lib.clomp_create.restype = ctypes.c_int
    lib.clomp_set_params.argtypes = [H, ctypes.POINTER(Params)]
    lib.clomp_set_params.restype = ctypes.c_int
    lib.clomp_solve_batch.argtypes = [H, ctypes.POINTER(Instance), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_void_p]
    lib.clomp_solve_batch.restype = ctypes.c_int
    lib.clomp_check_batch.argtypes = [H, ctypes.POINTER(Instance), ctypes.c_int32,
                                      ctypes.c_int32]
    lib.clomp_check_batch.restype = ctypes.c_int
    lib.clomp_grad.argtypes = [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_int32] + [ctypes.c_void_p] * 9
    lib.clomp_grad.restype = ctypes.c_int
    lib.clomp_grad_noalloc.argtypes = lib.clomp_grad.argtypes
    lib.clomp_grad_noalloc.restype = ctypes.c_int
    lib.clomp_profile_read.argtypes = [H, ctypes.POINTER(Profile)]
    lib.clomp_profile_read.restype = ctypes.c_int
    lib.clomp_profile_reset.argtypes = [H]
    lib.clomp_profile_reset.restype = ctypes.c_int
    lib.clomp_set_tuning.argtypes = [H, ctypes.POINTER(Tuning)]
    lib.clomp_set_tuning.restype = ctypes.c_int
    lib.clomp_get_tuning.argtypes = [H, ctypes.POINTER(Tuning)]
    lib.clomp_get_tuning.restype = ctypes.c_int
    lib.clomp_destroy.argtypes = [H]
    lib.clomp_destroy.restype = ctypes.c_int
    lib.clomp_status_string.argtypes = [ctypes.c_int]
    lib.clomp_status_string.restype = ctypes.c_char_p
    lib.clomp_last_error.argtypes = [H]
    lib.clomp_last_error.restype = ctypes.c_char_p
    lib.clomp_tuning_table_import.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
    lib.clomp_tuning_table_import.restype = ctypes.c_int
    lib.clomp_tuning_table_export.argtypes = [ctypes.c_char_p, ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_size_t)]
    lib.clomp_tuning_table_export.restype = ctypes.c_int
    lib.clomp_tuning_table_clear.argtypes = []
    lib.clomp_tuning_table_clear.restype = ctypes.c_int
    _lib = lib
    return lib


def default_params():
    p = Params()
    load_library().clomp_default_params(ctypes.byref(p))
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(h, rc, what):
    if rc != 0:
        lib = load_library()
        msg = lib.clomp_last_error(h).decode() if h else ""
        raise ClompError(f"{what}: {STATUS_NAMES.get(rc, rc)}: {msg}")


def dtype_code(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    if t.dtype == torch.float64:
        return F64
    raise ClompError(f"unsupported dtype {t.dtype}")


def _need(cond, msg):
    if not cond:
        raise ClompError(msg)


def _check_vec(name, t, device, dtypes, length):
    """A device vector of at least `length` contiguous elements."""
    _need(isinstance(t, torch.Tensor), f"{name} must be a tensor")
    _need(t.device == device, f"{name} is on {t.device}; the solver runs on {device}")
    _need(t.dtype in dtypes, f"{name} has dtype {t.dtype}; expected one of {dtypes}")
    _need(t.is_contiguous(), f"{name} must be contiguous")
    _need(t.numel() >= length, f"{name} has {t.numel()} elements; {length} are read")


def _check_atoms(name, t, device, dtypes, m, n=None):
    """An atom-major matrix (n, lda): unit stride along each atom, lda >= m,
    and storage for n * lda elements from its first element (the kernels read
    whole padded atoms)."""
    _need(isinstance(t, torch.Tensor), f"{name} must be a tensor")
    _need(t.device == device, f"{name} is on {t.device}; the solver runs on {device}")
    _need(t.dtype in dtypes, f"{name} has dtype {t.dtype}; expected one of {dtypes}")
    _need(t.dim() == 2 and (t.shape[1] <= 1 or t.stride(1) == 1),
          f"{name} must be 2-D (n, lda) with unit stride along each atom")
    _need(n is None or t.shape[0] == n, f"{name} has {t.shape[0]} atoms; expected {n}")
    lda = t.stride(0)
    _need(t.shape[1] >= m and lda >= m, f"{name}: lda = {lda} and width {t.shape[1]} must be "
                                        f">= m = {m}")
    extent = (t.storage_offset() + t.shape[0] * lda) * t.element_size()
    _need(t.untyped_storage().nbytes() >= extent,
          f"{name}: storage holds fewer than n * lda elements")


@dataclass
class BatchResult:
    x: list            # per instance: float32 tensor (n,)
    support: list      # per instance: int32 tensor (k,)
    n_selected: torch.Tensor
    resid_norm: torch.Tensor
    status: torch.Tensor


class Solver:
    """A library handle bound to one device, holding the solver parameters."""

    def __init__(self, device=0, method="clomp", inner_steps=None, lr_rel=0.05,
                 beta1=0.9, beta2=0.999, eps_rel=1e-8, refine_iters=0,
                 refine_tol=0.0, flags=0, select_threshold=0.7, prior_tv=0.0, prior_lv=0.0):
        lib = load_library()
        if not torch.cuda.is_available():
            raise ClompError("no GPU available: the CLOMP library runs only on the device")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        p = default_params()
        if method not in METHODS:
            raise ClompError(f"unknown method {method!r}")
        p.method = METHODS[method]
        if inner_steps is None:   # CLOMP: Adam steps per atom; IHT, paper mode: iterations
            inner_steps = 200 if method in ("iht", "clomp_paper") else 32
        p.inner_steps, p.lr_rel, p.beta1, p.beta2 = inner_steps, lr_rel, beta1, beta2
        p.eps_rel, p.refine_iters, p.refine_tol, p.flags = eps_rel, refine_iters, refine_tol, flags
        p.select_threshold = select_threshold
        p.prior_tv = prior_tv
        p.prior_lv = prior_lv
        self.params = p
        h = ctypes.c_void_p()
        _check(None, lib.clomp_create(ctypes.byref(h), self.device.index or 0, ctypes.byref(p)),
               "clomp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().clomp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        for key, v in kw.items():
            if key == "method":
                v = METHODS[v]
            setattr(self.params, key, v)
        _check(self._h, load_library().clomp_set_params(self._h, ctypes.byref(self.params)),
               "clomp_set_params")

    def set_tuning(self, scan_tile_kb=0, pass_tile_kb=0, team_min_rows=0, rscan_min_t=0,
                   shared_min_tiles=0, spin_limit=0):
        """0 keeps a value, -1 restores its default."""
        t = Tuning()
        t.scan_tile_kb, t.pass_tile_kb = scan_tile_kb, pass_tile_kb
        t.team_min_rows, t.rscan_min_t = team_min_rows, rscan_min_t
        t.shared_min_tiles, t.spin_limit = shared_min_tiles, spin_limit
        _check(self._h, load_library().clomp_set_tuning(self._h, ctypes.byref(t)),
               "clomp_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(self._h, load_library().clomp_get_tuning(self._h, ctypes.byref(t)),
               "clomp_get_tuning")
        return {"scan_tile_kb": t.scan_tile_kb, "pass_tile_kb": t.pass_tile_kb,
                "team_min_rows": t.team_min_rows, "rscan_min_t": t.rscan_min_t,
                "shared_min_tiles": t.shared_min_tiles, "spin_limit": t.spin_limit}

    def profile_reset(self):
        _check(self._h, load_library().clomp_profile_reset(self._h), "clomp_profile_reset")

    def profile_read(self):
        """Per-phase device time (ms) and launch counts since the last reset."""
        p = Profile()
        _check(self._h, load_library().clomp_profile_read(self._h, ctypes.byref(p)),
               "clomp_profile_read")
        return {"ms": {PHASES[i]: p.ms[i] for i in range(len(PHASES))},
                "launches": {PHASES[i]: int(p.launches[i]) for i in range(len(PHASES))},
                "scan_bytes": p.scan_bytes, "pass_bytes": p.pass_bytes,
                "fused_bytes": p.fused_bytes}

    # ------------------------------------------------------------------ solve
    def prepare(self, items, stream=None):
        """Pack the descriptors of a batch and allocate its outputs once (on the
        launch stream).  items: list of dicts with keys At (n, lda) float32 |
        bfloat16 cuda tensor, m, y (m,) float32, k, optional At_master
        (n, lda_master) float32.  `run` launches the batch; every run rewrites
        the same outputs."""
        count = len(items)
        dt = dtype_code(items[0]["At"]) if count else 0
        if any(dtype_code(it["At"]) != dt for it in items):
            raise ClompError("all instances of a batch must share the bulk dtype")
        dev = self.device
        # the library cannot see buffer sizes: every tensor is checked here,
        # before any launch
        seen = set()
        for q, it in enumerate(items):
            m = int(it["m"])
            _need(m > 0 and int(it["k"]) > 0, f"instance {q}: m and k must be positive")
            A = it["At"]
            if id(A) not in seen:
                _check_atoms(f"instance {q}: At", A, dev, (torch.float32, torch.bfloat16), m)
            Am = it.get("At_master")
            if Am is not None and id(Am) not in seen:
                _check_atoms(f"instance {q}: At_master", Am, dev, (torch.float32,), m,
                             n=A.shape[0])
                seen.add(id(Am))
            seen.add(id(A))
            _need(Am is not None or A.dtype == torch.float32,
                  f"instance {q}: a bfloat16 At needs a float32 At_master")
            _check_vec(f"instance {q}: y", it["y"], dev, (torch.float32,), m)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ns = np.fromiter((it["At"].shape[0] for it in items), np.int64, count)
        ks = np.fromiter((it["k"] for it in items), np.int64, count)
        xoff = np.concatenate(([0], np.cumsum(ns))).astype(np.int64)
        soff = np.concatenate(([0], np.cumsum(ks))).astype(np.int64)
        with torch.cuda.stream(st):
            x_all = torch.empty(int(xoff[-1]), dtype=torch.float32, device=dev)
            sup_all = torch.empty(int(soff[-1]), dtype=torch.int32, device=dev)
            nsel = torch.empty(count, dtype=torch.int32, device=dev)
            rnorm = torch.empty(count, dtype=torch.float64, device=dev)
            status = torch.empty(count, dtype=torch.int32, device=dev)
        arr = np.zeros(count, dtype=INSTANCE_NP)
        if count:
            arr["n"], arr["k"] = ns, ks
            arr["m"] = [int(it["m"]) for it in items]
            arr["lda"] = [it["At"].stride(0) for it in items]
            arr["A"] = [it["At"].data_ptr() for it in items]
            masters = [it.get("At_master") for it in items]
            arr["lda_master"] = [a.stride(0) if a is not None else 0 for a in masters]
            arr["A_master"] = [a.data_ptr() if a is not None else 0 for a in masters]
            arr["y"] = [it["y"].data_ptr() for it in items]
            arr["x"] = x_all.data_ptr() + 4 * xoff[:-1]
            arr["support"] = sup_all.data_ptr() + 4 * soff[:-1]
            idx = np.arange(count, dtype=np.int64)
            arr["n_selected"] = nsel.data_ptr() + 4 * idx
            arr["resid_norm"] = rnorm.data_ptr() + 8 * idx
            arr["status"] = status.data_ptr() + 4 * idx
        xs = [x_all[a:b] for a, b in zip(xoff[:-1].tolist(), xoff[1:].tolist())]
        sups = [sup_all[a:b] for a, b in zip(soff[:-1].tolist(), soff[1:].tolist())]
        return PreparedBatch(arr, count, dt, BatchResult(xs, sups, nsel, rnorm, status),
                             list(items), st, (x_all, sup_all, nsel, rnorm, status))

    def run(self, prep, stream=None):
        """Launch a prepared batch on `stream` (default: the stream it was
        prepared on); returns its BatchResult (the prepared output tensors)."""
        dev = self.device
        st = stream if stream is not None else prep.stream
        if prep.count == 0:
            return prep.result
        rc = load_library().clomp_solve_batch(
            self._h, prep.arr.ctypes.data_as(ctypes.POINTER(Instance)), prep.count, prep.dtype,
            ctypes.c_void_p(st.cuda_stream))
        _check(self._h, rc, "clomp_solve_batch")
        if st != torch.cuda.current_stream(dev) and st.cuda_stream not in prep.recorded:
            # tensors the caller may drop must outlive the queued work on `st`
            # (one record per stream: the allocator checks every recorded
            # stream when the tensor is freed)
            seen = set()
            for it in prep.items:
                for key in ("At", "At_master", "y"):
                    t = it.get(key)
                    if t is not None and id(t) not in seen:
                        seen.add(id(t))
                        t.record_stream(st)
            for t in prep.outputs:
                t.record_stream(st)
            prep.recorded.add(st.cuda_stream)
        self._keep = prep
        return prep.result

    def solve_batch(self, items, stream=None):
        """prepare + run for a one-off batch."""
        if len(items) == 0:
            return BatchResult([], [], *(torch.empty(0, device=self.device),) * 3)
        return self.run(self.prepare(items, stream), stream)

    def solve(self, At, m, y, k, At_master=None, stream=None):
        r = self.solve_batch([dict(At=At, m=m, y=y, k=k, At_master=At_master)], stream)
        return dict(x=r.x[0], support=r.support[0], n_selected=r.n_selected[0],
                    resid_norm=r.resid_norm[0], status=r.status[0])

    def solve_shared(self, At, m, Y, k, At_master=None, stream=None):
        """All rows of Y (a, m) share one matrix (the multi-signal model)."""
        items = [dict(At=At, m=m, y=Y[c], k=k, At_master=At_master) for c in range(Y.shape[0])]
        return self.solve_batch(items, stream)

    # ------------------------------------------------------------------ grad
    def grad(self, At, m, x, mask, y, grad_out=None, want_resid=True, stream=None,
             out=None, noalloc=False):
        """Returns (loss, grad_x, u) with u = A(mask*x) - y.  out: optional
        (loss, grad_x, u) tensors to write (u may be None).  noalloc: call
        clomp_grad_noalloc, whose scratch is the library's device-resident
        array (no allocation inside the call)."""
        dev = self.device
        kinds = (torch.float32, torch.float64)
        _check_atoms("At", At, dev, kinds, int(m))
        dt = dtype_code(At)
        n = int(At.shape[0])
        _check_vec("x", x, dev, (At.dtype,), n)
        _check_vec("y", y, dev, (At.dtype,), int(m))
        _check_vec("mask", mask, dev, (torch.uint8, torch.bool), n)
        if mask.dtype == torch.bool:
            mask = mask.view(torch.uint8)
        if grad_out is not None:
            _check_vec("grad_out", grad_out, dev, (At.dtype,), 1)
        if out is None:
            gx = torch.empty(n, dtype=At.dtype, device=dev)
            loss = torch.empty((), dtype=At.dtype, device=dev)
            u = torch.empty(m, dtype=At.dtype, device=dev) if want_resid else None
        else:
            loss, gx, u = out
            _check_vec("loss", loss, dev, (At.dtype,), 1)
            _check_vec("grad_x", gx, dev, (At.dtype,), n)
            if u is not None:
                _check_vec("u", u, dev, (At.dtype,), int(m))
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        lib = load_library()
        fn, name = ((lib.clomp_grad_noalloc, "clomp_grad_noalloc") if noalloc
                    else (lib.clomp_grad, "clomp_grad"))
        rc = fn(self._h, n, m, int(At.stride(0)), dt, _ptr(At), _ptr(x), _ptr(mask), _ptr(y),
                _ptr(grad_out), _ptr(gx), _ptr(u), _ptr(loss), ctypes.c_void_p(st.cuda_stream))
        _check(self._h, rc, name)
        return loss, gx, u


def _check_table(rc, what):
    if rc != 0:
        msg = load_library().clomp_last_error(None).decode()
        raise ClompError(f"{what}: {STATUS_NAMES.get(rc, rc)}: {msg}")


def tuning_table_import(text):
    """Merge a saved autotune table (the text of tuning_table_export) into the
    process-wide table; returns the number of entries."""
    n = ctypes.c_int32(0)
    _check_table(load_library().clomp_tuning_table_import(text.encode(), ctypes.byref(n)),
                 "clomp_tuning_table_import")
    return n.value


def tuning_table_export():
    """The process-wide autotune table as text."""
    lib = load_library()
    ln = ctypes.c_size_t(0)
    _check_table(lib.clomp_tuning_table_export(None, 0, ctypes.byref(ln)),
                 "clomp_tuning_table_export")
    buf = ctypes.create_string_buffer(ln.value + 1)
    _check_table(lib.clomp_tuning_table_export(buf, ln.value + 1, ctypes.byref(ln)),
                 "clomp_tuning_table_export")
    return buf.value.decode()


def tuning_table_clear():
    _check_table(load_library().clomp_tuning_table_clear(), "clomp_tuning_table_clear")


def save_tuning_table(path):
    with open(path, "w") as f:
        f.write(tuning_table_export())


def load_tuning_table(path):
    with open(path) as f:
        return tuning_table_import(f.read())


def check_batch(items_ctypes, count, dtype, handle=None):
    """Host-only validation (no HIP call); returns the status code."""
    return load_library().clomp_check_batch(handle, items_ctypes, count, dtype)


_default = {}


def solver_for(device=0, **kw):
    key = (device, tuple(sorted(kw.items())))
    if key not in _default:
        _default[key] = Solver(device, **kw)
    return _default[key]


class ClompLoss(torch.autograd.Function):
    """loss = 1/2 ||A(mask*x) - y||^2 with the hand-written HIP backward.

    forward(x, mask, At, m, y): At is (n, lda) atom-major, fixed (no gradient);
    mask is uint8 or bool (n,).  Gradients: grad_x = mask * A^T u * g,
    grad_y = -u * g.  The backward is not itself differentiable (a second
    derivative raises instead of returning zero).
    """

    @staticmethod
    def forward(ctx, x, mask, At, m, y):
        solver = solver_for(x.device.index or 0)
        loss, gx, u = solver.grad(At, m, x.contiguous(), mask.contiguous(), y.contiguous())
        ctx.save_for_backward(gx, u)
        return loss

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        gx, u = ctx.saved_tensors
        return gx * g, None, None, None, -u * g
