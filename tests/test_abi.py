"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/clomp.h, and validates arguments on the host before any
HIP call (clomp_check_batch never touches the device)."""

import ctypes
import os
import re

import pytest

from paper_2501_11592_amd import clomp as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clomp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clomp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(C.LIB_PATH):
        pytest.fail("libclomp.so is not built (run python -m paper_2501_11592_amd.build)")
    return C.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("clomp_create", "clomp_solve_batch", "clomp_grad", "clomp_destroy",
               "clomp_status_string", "clomp_last_error", "clomp_default_params",
               "clomp_check_batch", "clomp_set_params"):
        assert fn in names


def test_library_exports_every_declared_symbol(lib):
    for fn in declared_functions():
        assert hasattr(lib, fn), fn


def test_status_strings_and_defaults(lib):
    assert lib.clomp_status_string(0) == b"CLOMP_OK"
    assert lib.clomp_status_string(4) == b"CLOMP_NOT_SUPPORTED"
    p = C.Params()
    lib.clomp_default_params(ctypes.byref(p))
    assert p.method == 0 and p.inner_steps == 32
    assert abs(p.lr_rel - 0.05) < 1e-7 and abs(p.beta1 - 0.9) < 1e-7
    assert abs(p.beta2 - 0.999) < 1e-7 and p.resid_tol == 0.0
    assert abs(p.select_threshold - 0.7) < 1e-7 and p.prior_tv == 0.0 and p.prior_lv == 0.0


def header_struct_fields(name):
    """(field, element count) of `typedef struct { ... } name;` in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    out = []
    for decl in body.split(";"):
        for piece in decl.split(","):   # `int32_t n, m;` declares two fields
            mt = re.search(r"(\w+)\s*(?:\[(\d+)\])?\s*$", piece.strip())
            if mt:
                out.append((mt.group(1), int(mt.group(2) or 1)))
    return out


@pytest.mark.parametrize("name, cls", [("clomp_tuning_t", C.Tuning),
                                       ("clomp_params_t", C.Params),
                                       ("clomp_instance_t", C.Instance)])
def test_binding_structs_match_header(name, cls):
    """Field names, order and array lengths of the ctypes mirrors."""
    py = [(f[0], getattr(f[1], "_length_", 1)) for f in cls._fields_]
    assert py == header_struct_fields(name)


def test_tuning_struct_size():
    assert ctypes.sizeof(C.Tuning) == 8 * 4


def test_struct_layout_matches_header():
    assert ctypes.sizeof(C.Instance) == 4 * 4 + 2 * 8 + 8 * 8
    assert ctypes.sizeof(C.Params) == 13 * 4


def _inst(n=100, m=20, k=5, lda=20, A=4096, Am=0, ldm=0, y=8192):
    d = C.Instance()
    d.n, d.m, d.k, d.lda, d.lda_master = n, m, k, lda, ldm
    d.A, d.A_master, d.y = A, Am or None, y
    d.x, d.support, d.n_selected, d.resid_norm, d.status = 1 << 20, 2 << 20, 3 << 20, 4 << 20, 5 << 20
    return d


def _check(lib, insts, dtype=C.F32, count=None):
    arr = (C.Instance * max(1, len(insts)))(*insts)
    return lib.clomp_check_batch(None, arr, len(insts) if count is None else count, dtype)


def test_validation_accepts_well_formed(lib):
    assert _check(lib, [_inst()]) == 0
    assert _check(lib, [_inst(lda=24, A=16), _inst(n=3, m=3, k=9, lda=4)]) == 0
    assert _check(lib, [_inst(lda=32, Am=4096, ldm=20)], dtype=C.BF16) == 0
    assert _check(lib, [], count=0) == 0


@pytest.mark.parametrize("bad,code", [
    (dict(n=0), 1), (dict(m=-1), 1), (dict(k=0), 1),
    (dict(lda=19), 1),            # lda < m
    (dict(lda=22), 1),            # lda not a multiple of 4
    (dict(A=0), 1),               # NULL A
    (dict(A=4100), 1),            # misaligned A
    (dict(y=0), 1),               # NULL y
    (dict(k=3000, m=3000, n=3000, lda=3000), 4),   # k_eff beyond the Adam capacity
])
def test_validation_rejects(lib, bad, code):
    assert _check(lib, [_inst(**bad)]) == code


def test_validation_dtype_rules(lib):
    assert _check(lib, [_inst()], dtype=C.F64) == 4          # not served
    assert _check(lib, [_inst()], dtype=7) == 1              # unknown
    assert _check(lib, [_inst(lda=32)], dtype=C.BF16) == 1   # BF16 needs a master
    assert _check(lib, [_inst(lda=20)], dtype=C.BF16) == 1   # BF16 lda % 8
    assert _check(lib, [_inst(lda=32, Am=4098)], dtype=C.BF16) == 1  # misaligned master
    assert _check(lib, [_inst()], count=-1) == 1


def test_null_handle_and_null_out(lib):
    assert lib.clomp_create(None, 0, None) == 1
    assert lib.clomp_solve_batch(None, None, 0, 0, None) == 1
    assert lib.clomp_destroy(None) == 1
    assert lib.clomp_last_error(None) == b"no handle"


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(C, "_lib", None)
    with pytest.raises(C.ClompError):
        C.load_library(str(tmp_path / "missing.so"))


# ---- binding checks (no GPU needed: they run before any library call) ----
import torch  # noqa: E402

CPU = torch.device("cpu")


def _raises(fn, text):
    with pytest.raises(C.ClompError, match=text):
        fn()


def test_binding_rejects_matrices_the_kernels_would_overrun():
    ok = torch.zeros(10, 16)
    C._check_atoms("At", ok, CPU, (torch.float32,), 12)
    _raises(lambda: C._check_atoms("At", ok, CPU, (torch.float32,), 17), "must be >= m")
    _raises(lambda: C._check_atoms("At", ok.double(), CPU, (torch.float32,), 12), "dtype")
    _raises(lambda: C._check_atoms("At", ok.t(), CPU, (torch.float32,), 8), "unit stride")
    _raises(lambda: C._check_atoms("At", ok, CPU, (torch.float32,), 12, n=11), "atoms")
    # a (n, m) view of a padded buffer whose last atom's padding is missing
    buf = torch.zeros(10 * 16 - 4)
    view = buf.as_strided((10, 12), (16, 1))
    _raises(lambda: C._check_atoms("At", view, CPU, (torch.float32,), 12), "storage")
    full = torch.zeros(10 * 16).as_strided((10, 12), (16, 1))
    C._check_atoms("At", full, CPU, (torch.float32,), 12)
    _raises(lambda: C._check_atoms("At", ok, torch.device("meta"), (torch.float32,), 12),
            "solver runs on")


def test_binding_rejects_short_or_mistyped_vectors():
    y = torch.zeros(12)
    C._check_vec("y", y, CPU, (torch.float32,), 12)
    _raises(lambda: C._check_vec("y", y, CPU, (torch.float32,), 13), "13 are read")
    _raises(lambda: C._check_vec("y", y.double(), CPU, (torch.float32,), 12), "dtype")
    _raises(lambda: C._check_vec("y", torch.zeros(24)[::2], CPU, (torch.float32,), 12),
            "contiguous")
    _raises(lambda: C._check_vec("mask", torch.zeros(12, dtype=torch.int32), CPU,
                                 (torch.uint8, torch.bool), 12), "dtype")


def test_loss_backward_is_once_differentiable():
    fn = C.ClompLoss.backward
    assert getattr(fn, "__wrapped__", None) is not None or "once_differentiable" in repr(fn)


def test_set_tuning_ranges_documented_in_header():
    text = open(HEADER).read()
    assert "-1 restores the default" in text and "spin_limit" in text
