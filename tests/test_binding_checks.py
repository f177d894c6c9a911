"""The binding's argument checks, which run before any library call (the C
side cannot see buffer sizes): device, dtype, contiguity, length, the
atom-major layout of A and its storage extent.  CPU tensors checked against
the CPU device, so no GPU is needed."""

import pytest
import torch

from paper_2501_11592_amd import clomp as C

CPU = torch.device("cpu")
F32 = (torch.float32,)


def test_vector_checks():
    C._check_vec("y", torch.zeros(10), CPU, F32, 10)
    with pytest.raises(C.ClompError, match="must be a tensor"):
        C._check_vec("y", [0.0] * 10, CPU, F32, 10)
    with pytest.raises(C.ClompError, match="the solver runs on"):
        C._check_vec("y", torch.zeros(10), torch.device("cuda", 0), F32, 10)
    with pytest.raises(C.ClompError, match="dtype"):
        C._check_vec("y", torch.zeros(10, dtype=torch.float64), CPU, F32, 10)
    with pytest.raises(C.ClompError, match="contiguous"):
        C._check_vec("y", torch.zeros(20)[::2], CPU, F32, 10)
    with pytest.raises(C.ClompError, match="9 elements; 10 are read"):
        C._check_vec("y", torch.zeros(9), CPU, F32, 10)


def test_atom_major_checks():
    A = torch.zeros((100, 32))
    C._check_atoms("At", A, CPU, F32, 30, n=100)
    C._check_atoms("At", A[:, :30], CPU, F32, 30)          # a view: lda 32 >= m
    with pytest.raises(C.ClompError, match="2-D"):
        C._check_atoms("At", torch.zeros(3200), CPU, F32, 30)
    with pytest.raises(C.ClompError, match="unit stride"):
        C._check_atoms("At", torch.zeros((32, 100)).t(), CPU, F32, 30)
    with pytest.raises(C.ClompError, match="expected 99"):
        C._check_atoms("At", A, CPU, F32, 30, n=99)
    with pytest.raises(C.ClompError, match=">= m = 40"):
        C._check_atoms("At", A, CPU, F32, 40)
    with pytest.raises(C.ClompError, match="dtype"):
        C._check_atoms("At", A.double(), CPU, F32, 30)


def test_atom_storage_extent():
    """The kernels read n whole padded atoms (n * lda elements) from the first
    element: a narrow view that ends before its last atom's padding is
    refused, as is a view whose offset runs past the storage."""
    base = torch.zeros(100 * 32)
    A = base.as_strided((100, 30), (32, 1))                 # lda 32, storage 3200 elements
    C._check_atoms("At", A, CPU, F32, 30)
    short = torch.zeros(99 * 32 + 30).as_strided((100, 30), (32, 1))
    with pytest.raises(C.ClompError, match="fewer than n \\* lda"):
        C._check_atoms("At", short, CPU, F32, 30)
    shifted = base.as_strided((100, 30), (32, 1), storage_offset=2)
    with pytest.raises(C.ClompError, match="fewer than n \\* lda"):
        C._check_atoms("At", shifted, CPU, F32, 30)


def test_dtype_codes():
    assert C.dtype_code(torch.zeros(1)) == C.F32
    assert C.dtype_code(torch.zeros(1, dtype=torch.bfloat16)) == C.BF16
    assert C.dtype_code(torch.zeros(1, dtype=torch.float64)) == C.F64
    with pytest.raises(C.ClompError, match="unsupported dtype"):
        C.dtype_code(torch.zeros(1, dtype=torch.float16))
